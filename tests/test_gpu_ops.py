"""GPU parity of the operators against the CPU oracle, through the C ABI.

Small meshes span several workgroups with a ragged tail for every case
count; the full-size matvec workload (64^3 hexes x 6) is checked on sampled
nodes and by invariants.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import fem, solve, adjoint
from paper_1710_08679_amd import ebe, meshgen
from tests.helpers import (assert_close_bound, kappa_max, oracle_K, parity_mesh, restricted_matvec, sampled_matvec,
                           tol_factor)

pytestmark = pytest.mark.gpu

DT = {np.float64: torch.float64, np.float32: torch.float32}


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.fixture(scope="module")
def small(gpu_lib):
    m = parity_mesh(6, 5, 4, seed=1, bc=True)
    print(f"[parity mesh] E={m.n_elem} N={m.n_nodes}", flush=True)
    return m, ebe.Mesh.from_generated(m), oracle_K(m), oracle_K(m, order=1), kappa_max(m)


FORMS = [ebe.FORM_GATHER, ebe.FORM_STAGED, ebe.FORM_PIPELINED, ebe.FORM_COLOURED,
         ebe.FORM_DETERMINISTIC]  # quadratic level
FORMS1 = [ebe.FORM_GATHER, ebe.FORM_STAGED, ebe.FORM_PIPELINED, ebe.FORM_ASSEMBLED]  # linear level
# second variants: pipelined and coloured kernels with the geometry read per
# work-item, gather and staged kernels with the geometry formed from the corners,
# the deterministic form colour by colour, the assembled form in its other tiles
FORMS_V = FORMS + [(ebe.FORM_PIPELINED, 1), (ebe.FORM_COLOURED, 1), (ebe.FORM_GATHER, 1), (ebe.FORM_STAGED, 1),
                   (ebe.FORM_DETERMINISTIC, 1)]
FORMS1_V = FORMS1 + [(ebe.FORM_PIPELINED, 1), (ebe.FORM_GATHER, 1), (ebe.FORM_ASSEMBLED, 1), (ebe.FORM_ASSEMBLED, 2)]


class forced_form:
    """Run the products of one (level, dtype, nrhs) in a given form."""

    def __init__(self, gm, level, dtype, nrhs, form):
        form, variant = form if isinstance(form, tuple) else (form, 0)
        self.args = (gm, level, DT[dtype], nrhs, form)
        self.variant = variant

    def __enter__(self):
        gm, level, dt, nrhs, form = self.args
        gm.set_form(level, dt, nrhs, form)
        gm.set_variant(level, dt, nrhs, self.variant)
        assert gm.form(level, dt, nrhs) == form and gm.variant(level, dt, nrhs) == self.variant

    def __exit__(self, *exc):
        gm, level, dt, nrhs, _ = self.args
        gm.set_form(level, dt, nrhs, ebe.FORM_AUTO)  # (resets the variant too)


@pytest.mark.parametrize("form", FORMS_V)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [1, 2, 3, 4, 7, 9, 16])
def test_matvec_matches_oracle(small, dtype, nrhs, form):
    m, gm, K, _, kap = small
    x = meshgen.rng_for(80, nrhs).standard_normal((m.n_nodes, 3, nrhs))
    xd = x.astype(dtype)
    with forced_form(gm, 0, dtype, nrhs, form):
        y = gm.matvec(to_dev(xd, dtype)).cpu().numpy().astype(np.float64)
    ref = (K @ xd.astype(np.float64).reshape(-1, nrhs)).reshape(y.shape)
    assert_close_bound(y, ref, abs(K), xd.astype(np.float64), dtype, kap,
                       f"matvec {dtype.__name__} n={nrhs} form={form}")


@pytest.mark.parametrize("form", FORMS_V)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [5, 6, 8, 10, 11, 12, 13, 14, 15])
def test_matvec_other_case_counts(small, dtype, nrhs, form):
    """The case counts the test above leaves out: each is its own kernel
    instantiation, with its own pass widths and vector widths."""
    m, gm, K, _, kap = small
    x = meshgen.rng_for(86, nrhs).standard_normal((m.n_nodes, 3, nrhs)).astype(dtype)
    with forced_form(gm, 0, dtype, nrhs, form):
        y = gm.matvec(to_dev(x, dtype), apply_bc=True).cpu().numpy().astype(np.float64)
    xr = x.astype(np.float64)
    assert_close_bound(y, fem.matvec_bc(K, xr, m.fixed), abs(K), xr, dtype, kap,
                       f"P K P x {dtype.__name__} n={nrhs} form={form}")


@pytest.mark.parametrize("form", FORMS_V)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_matvec_with_dirichlet_projection(small, dtype, form):
    m, gm, K, _, kap = small
    x = meshgen.rng_for(81, 0).standard_normal((m.n_nodes, 3, 5)).astype(dtype)
    with forced_form(gm, 0, dtype, 5, form):
        y = gm.matvec(to_dev(x, dtype), apply_bc=True).cpu().numpy().astype(np.float64)
    ref = fem.matvec_bc(K, x.astype(np.float64), m.fixed)
    assert np.all(y[m.fixed.astype(bool)] == 0.0)
    assert_close_bound(y, ref, abs(K), x.astype(np.float64), dtype, kap, "matvec P K P")


@pytest.mark.parametrize("form", FORMS1_V)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16])
def test_linear_matvec_matches_oracle(small, dtype, form, nrhs):
    m, gm, _, K1, kap = small
    x = meshgen.rng_for(82, nrhs).standard_normal((m.n_vertices, 3, nrhs)).astype(dtype)
    with forced_form(gm, 1, dtype, nrhs, form):
        y = gm.matvec_p1(to_dev(x, dtype)).cpu().numpy().astype(np.float64)
        yb = gm.matvec_p1(to_dev(x, dtype), apply_bc=True).cpu().numpy().astype(np.float64)
    ref = (K1 @ x.astype(np.float64).reshape(-1, nrhs)).reshape(y.shape)
    assert_close_bound(y, ref, abs(K1), x.astype(np.float64), dtype, kap, "K1 x")
    refb = fem.matvec_bc(K1, x.astype(np.float64), m.fixed[:m.n_vertices])
    assert_close_bound(yb, refb, abs(K1), x.astype(np.float64), dtype, kap, "P K1 P x")


@pytest.mark.parametrize("form", FORMS_V)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("apply_bc", [False, True])
def test_matvec_add_accumulates(small, dtype, form, apply_bc):
    """y += K x (or P K P x): exclusive nodes add in the patch kernel, shared
    nodes in the shared-node pass; fixed DOFs of y keep their value."""
    m, gm, K, _, kap = small
    x = meshgen.rng_for(84, 0).standard_normal((m.n_nodes, 3, 6)).astype(dtype)
    y0 = meshgen.rng_for(84, 1).standard_normal((m.n_nodes, 3, 6)).astype(dtype)
    yd = to_dev(y0, dtype)
    with forced_form(gm, 0, dtype, 6, form):
        gm.matvec_add(to_dev(x, dtype), yd, apply_bc=apply_bc)
    y = yd.cpu().numpy().astype(np.float64)
    xr = x.astype(np.float64)
    Kx = fem.matvec_bc(K, xr, m.fixed) if apply_bc else (K @ xr.reshape(-1, 6)).reshape(y.shape)
    ref = y0.astype(np.float64) + Kx
    if apply_bc:
        fixed = m.fixed.astype(bool)
        assert np.array_equal(y[fixed], y0.astype(np.float64)[fixed])
    u = np.finfo(dtype).eps / 2
    bound = tol_factor(dtype, kap) * (abs(K) @ np.abs(xr).reshape(-1, 6)).reshape(y.shape) + 4 * u * np.abs(ref)
    assert np.all(np.abs(y - ref) <= bound), float(np.max(np.abs(y - ref) / bound))


def test_autotune_keeps_the_faster_form(small):
    m, gm, K, _, kap = small
    for level, nrhs in ((0, 4), (1, 16)):
        ts = gm.autotune(level, torch.float32, nrhs)
        print(f"[autotune level {level} n={nrhs}] ms by form: {ts}", flush=True)
        have = [t for t in ts if t >= 0]
        assert len(ts) == ebe.NUM_FORMS and min(have) > 0
        assert len(have) == (5 if level == 0 else 4)
        if level == 0:
            assert ts[ebe.FORM_ASSEMBLED] == -1
        else:
            assert ts[ebe.FORM_COLOURED] == -1 and ts[ebe.FORM_DETERMINISTIC] == -1
        assert gm.form(level, torch.float32, nrhs) == ts.index(min(have))
        gm.set_form(level, torch.float32, nrhs, ebe.FORM_AUTO)
    with pytest.raises(ebe.EbeError):
        gm.set_form(0, torch.float32, 4, 7)
    with pytest.raises(ebe.EbeError):
        gm.set_form(0, torch.float32, 4, ebe.FORM_ASSEMBLED)
    with pytest.raises(ebe.EbeError):
        gm.set_form(1, torch.float32, 4, ebe.FORM_COLOURED)
    with pytest.raises(ebe.EbeError):
        gm.set_form(1, torch.float32, 4, ebe.FORM_DETERMINISTIC)
    with pytest.raises(ebe.EbeError):
        gm.autotune(2, torch.float32, 4)


def test_multi_rhs_equals_single_columns(small):
    m, gm, K, _, kap = small
    x = to_dev(meshgen.rng_for(83, 0).standard_normal((m.n_nodes, 3, 16)), np.float64)
    y = gm.matvec(x)
    for j in (0, 5, 15):
        yj = gm.matvec(x[:, :, j:j + 1].contiguous())
        assert torch.allclose(yj[:, :, 0], y[:, :, j], rtol=0, atol=1e-13 * float(y.abs().max()))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [3, 6, 16])
def test_grid_transfers_match_oracle(small, dtype, nrhs):
    m, gm, _, _, kap = small
    P = fem.prolongation_p1(m.conn, m.n_nodes, m.n_vertices)
    xc = meshgen.rng_for(84, 0).standard_normal((m.n_vertices, 3, nrhs)).astype(dtype)
    xf = meshgen.rng_for(84, 1).standard_normal((m.n_nodes, 3, nrhs)).astype(dtype)
    yp = gm.prolong(to_dev(xc, dtype)).cpu().numpy().astype(np.float64)
    yr = gm.restrict(to_dev(xf, dtype)).cpu().numpy().astype(np.float64)
    rp = fem.apply_scalar_op(P, xc.astype(np.float64))
    rr = fem.apply_scalar_op(P.T.tocsr(), xf.astype(np.float64))
    u = float(np.finfo(dtype).eps)
    assert np.max(np.abs(yp - rp)) <= 2 * u * np.max(np.abs(rp))
    assert np.max(np.abs(yr - rr)) <= 16 * u * np.max(np.abs(rr))
    ybc = gm.prolong(to_dev(xc, dtype), apply_bc=True).cpu().numpy()
    assert np.all(ybc[m.fixed.astype(bool)] == 0)
    yrb = gm.restrict(to_dev(xf, dtype), apply_bc=True).cpu().numpy()
    assert np.all(yrb[m.fixed[:m.n_vertices].astype(bool)] == 0)


def test_diag_blocks_and_block_jacobi_match_oracle(small):
    m, gm, K, K1, kap = small
    for level, KK, fx, rows in ((0, K, m.fixed, m.n_nodes), (1, K1, m.fixed[:m.n_vertices], m.n_vertices)):
        got = gm.diag_blocks(level).cpu().numpy()
        ref = fem.diag_blocks(KK, rows)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
        Minv = solve.block_jacobi_inverse(KK, fx, rows)
        x = meshgen.rng_for(85, level).standard_normal((rows, 3, 4))
        x[fx.astype(bool)] = 0.0
        z = gm.block_jacobi(to_dev(x, np.float64), level).cpu().numpy()
        zr = np.einsum("nab,nbr->nar", Minv, x)
        assert np.max(np.abs(z - zr)) <= 1e-12 * np.max(np.abs(zr))
        z32 = gm.block_jacobi(to_dev(x, np.float32), level).cpu().numpy()
        assert np.max(np.abs(z32 - zr)) <= 1e-5 * np.max(np.abs(zr))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [1, 3, 4])
def test_adjoint_element_gradient_matches_oracle(small, dtype, nrhs):
    m, gm, _, _, kap = small
    rng = meshgen.rng_for(86, nrhs)
    u = rng.standard_normal((m.n_nodes, 3, nrhs))
    lam = rng.standard_normal((m.n_nodes, 3, nrhs))
    u[m.fixed.astype(bool)] = 0
    lam[m.fixed.astype(bool)] = 0
    ref = adjoint.element_gradient(m.xyz, m.conn, m.poisson, u, lam)
    g = gm.adjoint_grad(to_dev(u, dtype), to_dev(lam, dtype)).cpu().numpy().astype(np.float64)
    tol = (1e-12 if dtype == np.float64 else 2e-5) * np.max(np.abs(ref))
    assert np.max(np.abs(g - ref)) <= tol


def test_argument_errors(small):
    m, gm, _, _, kap = small
    x = torch.zeros((m.n_nodes, 3, 17), dtype=torch.float64, device="cuda")
    with pytest.raises(ebe.EbeError) as ei:
        gm.matvec(x)
    assert ei.value.status == ebe.ERR_ARG
    x = torch.zeros((m.n_nodes, 3, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(ebe.EbeError):
        gm.matvec(x, out=x)
    y = gm.matvec(x)
    assert float(y.abs().max()) == 0.0
    # a vector that is not 16-byte aligned is refused before any launch
    lib = ebe.load()
    big = torch.zeros(m.n_nodes * 6 + 2, dtype=torch.float64, device="cuda")
    st = lib.ebe_matvec(gm.handle, ebe.F64, 2, ctypes.c_void_p(big.data_ptr() + 8),
                        ctypes.c_void_p(y.data_ptr()), 0, None)
    assert st == ebe.ERR_ARG
    assert b"aligned" in lib.ebe_last_error()


def test_single_element_mesh(gpu_lib):
    m = meshgen.kuhn_mesh(1, 1, 1)
    keep = m.conn[:1]
    used = np.unique(keep)
    vmap = -np.ones(m.n_nodes, dtype=np.int64)
    verts = used[used < m.n_vertices]
    edges = used[used >= m.n_vertices]
    vmap[verts] = np.arange(verts.size)
    vmap[edges] = verts.size + np.arange(edges.size)
    conn = vmap[keep].astype(np.int32)
    xyz = np.zeros((used.size, 3))
    xyz[vmap[used]] = m.xyz[used]
    gm = ebe.Mesh(xyz, conn, 4, np.array([2.0]), np.array([0.3]))
    x = meshgen.rng_for(87, 0).standard_normal((10, 3, 2))
    y = gm.matvec(to_dev(x, np.float64)).cpu().numpy()
    Ke = fem.element_stiffness_p2(xyz[conn[0]][None], np.array([2.0]), np.array([0.3]))[0]
    ref = (Ke @ x[conn[0]].reshape(30, 2)).reshape(10, 3, 2)
    assert np.max(np.abs(y[conn[0]] - ref)) <= 1e-13 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# full-size matvec workload: 64^3 hexes x 6 tets, 3 layers, jitter 0.2h
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def big(gpu_lib):
    m = meshgen.matvec_mesh(64)
    print(f"[matvec workload] E={m.n_elem} N={m.n_nodes}", flush=True)
    return m, ebe.Mesh.from_generated(m), kappa_max(m)


@pytest.mark.parametrize("form", FORMS + [(ebe.FORM_GATHER, 1), (ebe.FORM_DETERMINISTIC, 1), "tuned"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [1, 16])
def test_full_size_matvec_sampled_nodes(big, dtype, nrhs, form):
    """The 64^3 workload in every product form and in the form the autotuner
    picks (the configuration bench.py times), on sampled nodes.  At 16 cases
    the staged shared-node partials (616 MB FP32, 1.2 GB FP64) exceed the
    256 MB last-level cache and take the streamed (non-temporal) path; at one
    case they do not."""
    m, gm, kap = big
    x = meshgen.random_vectors(meshgen.rng_for(2, 10 + nrhs), m.n_nodes, nrhs)
    xd = x.astype(dtype)
    if form == "tuned":
        gm.autotune(0, DT[dtype], nrhs)
        y = gm.matvec(to_dev(xd, dtype)).cpu().numpy().astype(np.float64)
        gm.set_form(0, DT[dtype], nrhs, ebe.FORM_AUTO)
    else:
        with forced_form(gm, 0, dtype, nrhs, form):
            y = gm.matvec(to_dev(xd, dtype)).cpu().numpy().astype(np.float64)
    nodes = meshgen.rng_for(2, 50).choice(m.n_nodes, size=96, replace=False)
    nodes = np.concatenate([nodes, [0, m.n_vertices - 1, m.n_vertices, m.n_nodes - 1]])
    ref, bnd = sampled_matvec(m, xd.astype(np.float64), nodes)
    tol = tol_factor(dtype, kap) * bnd
    err = np.abs(y[nodes] - ref)
    assert np.all(err <= tol), float(np.max(err / tol))


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("dtype,nrhs", [(np.float32, 16), (np.float64, 7), (np.float32, 1)])
def test_deterministic_form_is_bitwise_reproducible(big, dtype, nrhs, variant):
    """The deterministic form on the 64^3 workload: repeated products, with
    products of the other forms launched in between (other schedules, other
    cache contents), give the same bits; and they match the oracle on
    sampled nodes (the parity tests above cover it on every mesh)."""
    m, gm, kap = big
    x = to_dev(meshgen.random_vectors(meshgen.rng_for(2, 40 + nrhs), m.n_nodes, nrhs), dtype)
    outs = []
    for rep in range(4):
        with forced_form(gm, 0, dtype, nrhs, (ebe.FORM_DETERMINISTIC, variant)):
            outs.append(gm.matvec(x, apply_bc=rep % 2 == 0))
        with forced_form(gm, 0, dtype, nrhs, FORMS[rep % 4]):
            gm.matvec(x)
    assert torch.equal(outs[0], outs[2]) and torch.equal(outs[1], outs[3])
    with forced_form(gm, 0, dtype, nrhs, ebe.FORM_COLOURED):
        other = [gm.matvec(x) for _ in range(2)]
    print(f"[deterministic n={nrhs}] coloured form repeats equal: {torch.equal(other[0], other[1])}", flush=True)


def test_full_size_matvec_invariants(big):
    m, gm, _ = big
    x = to_dev(meshgen.random_vectors(meshgen.rng_for(2, 30), m.n_nodes, 4), np.float64)
    y = gm.matvec(x)
    # translations are in the kernel of K: 1^T (K x)_c = 0 for every component and case
    s = y.sum(dim=0)
    assert float(s.abs().max()) <= 1e-9 * float(y.abs().sum(dim=0).max())
    # symmetry: (x_a, K x_b) = (x_b, K x_a)
    a, b = x[:, :, 0:1].contiguous(), x[:, :, 1:2].contiguous()
    lhs = float((a * gm.matvec(b)).sum())
    rhs = float((b * gm.matvec(a)).sum())
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    # rigid rotation field gives zero force everywhere
    X = torch.from_numpy(m.xyz).cuda()
    rot = torch.stack([-X[:, 1], X[:, 0], torch.zeros_like(X[:, 0])], dim=1)[:, :, None].contiguous()
    yr = gm.matvec(rot)
    assert float(yr.abs().max()) <= 1e-10 * float(gm.matvec(x[:, :, :1].contiguous()).abs().max())


def test_full_size_f32_n16_tuned_at_xcd_range_boundaries(big):
    """The benchmarked configuration (FP32, 16 cases, the tuned form) checked at
    every node of whole patches where the patch kernels change hands: the
    first patches, the first, second and last patches of each XCD's contiguous
    range (a 2x2x2-hex block of 48 elements per patch on this Morton-ordered
    mesh), the patches a persistent workgroup reaches on its second trip, and
    the last patches."""
    m, gm, kap = big
    nrhs = 16
    x = meshgen.random_vectors(meshgen.rng_for(2, 40), m.n_nodes, nrhs).astype(np.float32)
    gm.autotune(0, torch.float32, nrhs)
    try:
        y = gm.matvec(to_dev(x, np.float32)).cpu().numpy().astype(np.float64)
    finally:
        gm.set_form(0, torch.float32, nrhs, ebe.FORM_AUTO)
    npatch = m.n_elem // 48
    q = npatch // 8
    patches = set()
    for xcd in range(9):
        for d in (-2, -1, 0, 1, 63, 64, 65, 130):
            p = xcd * q + d
            if 0 <= p < npatch:
                patches.add(p)
    els = np.concatenate([np.arange(48 * p, 48 * p + 48) for p in sorted(patches)])
    nodes = np.unique(m.conn[els])
    print(f"[xcd boundaries] {len(patches)} patches, {nodes.size} nodes", flush=True)
    ref, bnd = restricted_matvec(m, x.astype(np.float64), nodes)
    tol = tol_factor(np.float32, kap) * bnd
    err = np.abs(y[nodes] - ref)
    assert np.all(err <= tol), float(np.max(err / tol))


@pytest.mark.parametrize("form", FORMS + ["tuned"])
def test_full_size_f32_n16_all_nodes_against_fp64(big, form):
    """Every node of the FP32 16-case product against the FP64 product of the
    same (FP32-rounded) input: a lost or doubled partial sum anywhere would be
    an O(1) error at its node."""
    m, gm, kap = big
    nrhs = 16
    x = meshgen.random_vectors(meshgen.rng_for(2, 41), m.n_nodes, nrhs).astype(np.float32)
    xd = to_dev(x, np.float32)
    y64 = gm.matvec(xd.double())
    if form == "tuned":
        gm.autotune(0, torch.float32, nrhs)
        y32 = gm.matvec(xd)
        gm.set_form(0, torch.float32, nrhs, ebe.FORM_AUTO)
    else:
        with forced_form(gm, 0, np.float32, nrhs, form):
            y32 = gm.matvec(xd)
    err = (y32.double() - y64).abs()
    scale = float(y64.abs().max())
    assert float(err.max()) <= 2e-4 * scale, float(err.max()) / scale
    assert float(err.norm() / y64.norm()) <= 1e-5


# ---------------------------------------------------------------------------
# unordered numbering: elements and node ids shuffled (vertex-first kept)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def shuffled(gpu_lib):
    m = meshgen.shuffled(parity_mesh(5, 4, 4, seed=3, bc=True), meshgen.rng_for(78, 0))
    print(f"[shuffled parity mesh] E={m.n_elem} N={m.n_nodes}", flush=True)
    return m, ebe.Mesh.from_generated(m), oracle_K(m), oracle_K(m, order=1), kappa_max(m)


@pytest.mark.parametrize("form", FORMS_V)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [1, 4, 16])
def test_shuffled_mesh_matvec_matches_oracle(shuffled, dtype, nrhs, form):
    """Consecutive elements of a shuffled mesh share few nodes, so patches are
    cut by the node limit long before the element limit and most of their
    nodes are shared with other patches."""
    m, gm, K, _, kap = shuffled
    x = meshgen.rng_for(79, nrhs).standard_normal((m.n_nodes, 3, nrhs)).astype(dtype)
    with forced_form(gm, 0, dtype, nrhs, form):
        y = gm.matvec(to_dev(x, dtype)).cpu().numpy().astype(np.float64)
        yb = gm.matvec(to_dev(x, dtype), apply_bc=True).cpu().numpy().astype(np.float64)
    xr = x.astype(np.float64)
    ref = (K @ xr.reshape(-1, nrhs)).reshape(y.shape)
    assert_close_bound(y, ref, abs(K), xr, dtype, kap, f"shuffled K x {dtype.__name__} n={nrhs} form={form}")
    assert_close_bound(yb, fem.matvec_bc(K, xr, m.fixed), abs(K), xr, dtype, kap, "shuffled P K P x")


@pytest.mark.parametrize("form", FORMS1_V)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_shuffled_mesh_linear_matvec_matches_oracle(shuffled, dtype, form):
    m, gm, _, K1, kap = shuffled
    x = meshgen.rng_for(79, 100).standard_normal((m.n_vertices, 3, 7)).astype(dtype)
    with forced_form(gm, 1, dtype, 7, form):
        y = gm.matvec_p1(to_dev(x, dtype)).cpu().numpy().astype(np.float64)
    xr = x.astype(np.float64)
    ref = (K1 @ xr.reshape(-1, 7)).reshape(y.shape)
    assert_close_bound(y, ref, abs(K1), xr, dtype, kap, f"shuffled K1 x form={form}")


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_coloured_form_on_unordered_patches(shuffled, dtype, variant):
    """The coloured form on a shuffled mesh (patches cut by the node limit,
    most of their nodes shared, so most colours and most read-modify-write
    entries): P K P x against the oracle on repeated products, and the
    patch colouring's counts."""
    m, gm, K, _, kap = shuffled
    info = gm.patch_info(0)
    print(f"[shuffled patches] {info}", flush=True)
    assert info["colours"] >= 2 and info["patches"] >= info["colours"] and info["staged"] >= info["shared"]
    x = to_dev(meshgen.rng_for(79, 200).standard_normal((m.n_nodes, 3, 5)), dtype)
    xr = x.cpu().numpy().astype(np.float64)
    with forced_form(gm, 0, dtype, 5, (ebe.FORM_COLOURED, variant)):
        for _ in range(3):
            y = gm.matvec(x, apply_bc=True).cpu().numpy().astype(np.float64)
            assert_close_bound(y, fem.matvec_bc(K, xr, m.fixed), abs(K), xr, dtype, kap, "coloured P K P x")

