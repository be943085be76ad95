"""Curved (isoparametric) 10-node tetrahedra on the GPU against the oracle,
through the C ABI (``ebe_mesh_create_curved``; Section 2, Eq. (2) with the
Jacobian evaluated at each quadrature point).

* y = K x (and P K P x, y += K x, the allocation-free entry point) on a
  randomly curved mesh, elementwise within c * kappa * u * (|K| |x|), kappa
  the largest condition number of the quadrature-point Jacobians, n in
  {1, 4, 7, 16}, FP64 and FP32.
* The curved kernel on straight elements equals the straight-sided kernel to
  the same bound.
* A quadratically mapped lattice: K applied to a linear field vanishes at
  interior nodes (an oracle-free invariant that holds at any size).
* Quadratic-level diagonal blocks and block Jacobi against the oracle's.
* Algorithm 1 (mixed MG3, FP64) on a curved crust against the oracle's sparse
  direct solve.
* Entry points that need straight elements refuse curved meshes.
"""
import numpy as np
import pytest
import torch

from oracle import fem, solve
from paper_1710_08679_amd import ebe, meshgen
from tests.helpers import C_TOL, oracle_K, parity_mesh, unit_roundoff

pytestmark = pytest.mark.gpu

DT = {np.float64: torch.float64, np.float32: torch.float32}


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def kappa_points(m):
    """Largest 2-norm condition number of the Jacobians at the 4 quadrature
    points of every element (the geometry the kernel inverts)."""
    pts, _ = fem.tet_rule_4()
    xe = m.xyz[m.conn]
    kap = 0.0
    for q in range(len(pts)):
        _, dN = fem.p2_shape(pts[q])
        J = np.einsum("mna,nd->mad", xe, dN)
        s = np.linalg.svd(J, compute_uv=False)
        kap = max(kap, float(np.max(s[:, 0] / s[:, 2])))
    return kap


def check_bound(got, ref, absK, x, dtype, kappa, what):
    N, _, n = x.shape
    bound = (absK @ np.abs(x).reshape(3 * N, n)).reshape(got.shape)
    tol = C_TOL[dtype] * kappa * unit_roundoff(dtype) * bound + 1e-300
    worst = float(np.max(np.abs(got - ref) / tol))
    assert worst <= 1.0, f"{what}: max |err| / bound = {worst:.3g}"


@pytest.fixture(scope="module")
def curved(gpu_lib):
    base = parity_mesh(6, 5, 4, seed=3, bc=True)
    m = meshgen.curve_edges(base, meshgen.rng_for(78, 1), amp=0.06)
    gm = ebe.Mesh.from_generated(m, curved=True)
    K = oracle_K(m)
    kap = kappa_points(m)
    print(f"[curved parity mesh] E={m.n_elem} N={m.n_nodes} kappa={kap:.3g}", flush=True)
    return m, gm, K, abs(K), kap


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [1, 2, 4, 7, 16])
def test_curved_matvec_matches_oracle(curved, dtype, nrhs):
    m, gm, K, absK, kap = curved
    x = meshgen.random_vectors(meshgen.rng_for(79, nrhs), m.n_nodes, nrhs).astype(dtype).astype(np.float64)
    y = gm.matvec(to_dev(x, dtype)).cpu().numpy().astype(np.float64)
    ref = (K @ x.reshape(-1, nrhs)).reshape(x.shape)
    check_bound(y, ref, absK, x, dtype, kap, f"y = K x n={nrhs}")
    # P K P x
    yb = gm.matvec(to_dev(x, dtype), apply_bc=True).cpu().numpy().astype(np.float64)
    xm = fem.mask_fixed(x, m.fixed)
    refb = fem.mask_fixed((K @ xm.reshape(-1, nrhs)).reshape(x.shape), m.fixed)
    check_bound(yb, refb, absK, xm, dtype, kap, f"P K P x n={nrhs}")
    # y += K x: the bound of the product plus the rounding of the final sum
    y0 = meshgen.random_vectors(meshgen.rng_for(80, nrhs), m.n_nodes, nrhs).astype(dtype)
    ya = to_dev(y0, dtype)
    gm.matvec_add(to_dev(x, dtype), ya)
    refa = y0.astype(np.float64) + ref
    bound = (C_TOL[dtype] * kap * unit_roundoff(dtype) * (absK @ np.abs(x).reshape(-1, nrhs)).reshape(x.shape)
             + 4 * unit_roundoff(dtype) * np.abs(refa))
    err = np.abs(ya.cpu().numpy().astype(np.float64) - refa)
    assert np.all(err <= bound), float(np.max(err / bound))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_curved_noalloc_matches_matvec(curved, dtype):
    m, gm, K, absK, kap = curved
    for nrhs in (16, 3):  # two calls in a row, the second smaller
        x = to_dev(meshgen.random_vectors(meshgen.rng_for(81, nrhs), m.n_nodes, nrhs, dtype=dtype), dtype)
        a = gm.matvec(x, apply_bc=True)
        b = gm.matvec_noalloc(x, apply_bc=True)
        ref = (K @ fem.mask_fixed(x.cpu().numpy().astype(np.float64), m.fixed).reshape(-1, nrhs))
        ref = fem.mask_fixed(ref.reshape(m.n_nodes, 3, nrhs), m.fixed)
        xm = fem.mask_fixed(x.cpu().numpy().astype(np.float64), m.fixed)
        check_bound(b.cpu().numpy().astype(np.float64), ref, absK, xm, dtype, kap, "noalloc")
        check_bound(a.cpu().numpy().astype(np.float64), ref, absK, xm, dtype, kap, "matvec")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_curved_kernel_on_straight_elements_equals_straight_kernel(gpu_lib, dtype):
    m = parity_mesh(5, 4, 4, seed=4)
    gs = ebe.Mesh.from_generated(m)
    gc = ebe.Mesh.from_generated(m, curved=True)
    K = oracle_K(m)
    x = meshgen.random_vectors(meshgen.rng_for(82, 0), m.n_nodes, 5).astype(dtype).astype(np.float64)
    ys = gs.matvec(to_dev(x, dtype)).cpu().numpy().astype(np.float64)
    yc = gc.matvec(to_dev(x, dtype)).cpu().numpy().astype(np.float64)
    check_bound(yc, ys, abs(K), x, dtype, 2 * kappa_points(m), "curved vs straight kernel")


def test_mapped_lattice_linear_field_equilibrated_on_gpu(gpu_lib):
    m = meshgen.quadratic_map(meshgen.kuhn_mesh(10, 10, 10, jitter=0.2, rng=meshgen.rng_for(83, 0)), 0.3)
    gm = ebe.Mesh.from_generated(m, curved=True)
    A = meshgen.rng_for(83, 1).standard_normal((3, 3, 4))
    u = np.einsum("nd,cdr->ncr", m.xyz, A)
    y = gm.matvec(to_dev(u, np.float64)).cpu().numpy()
    r = m.refined
    inner = np.all((r > 0) & (r < 2 * np.array(m.grid)), axis=1)
    scale = np.abs(y).max()
    print(f"[mapped lattice] interior max {np.abs(y[inner]).max() / scale:.3g} of the boundary forces", flush=True)
    assert np.abs(y[inner]).max() <= 1e-11 * scale
    assert np.abs(y[~inner]).max() > 1e-3 * scale


def test_curved_diag_blocks_and_block_jacobi_match_oracle(curved):
    m, gm, K, absK, kap = curved
    got = gm.diag_blocks(0).cpu().numpy()
    ref = fem.diag_blocks(K, m.n_nodes)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    Minv = solve.block_jacobi_inverse(K, m.fixed, m.n_nodes)
    x = meshgen.rng_for(84, 0).standard_normal((m.n_nodes, 3, 4))
    x[m.fixed.astype(bool)] = 0.0
    z = gm.block_jacobi(to_dev(x, np.float64), 0).cpu().numpy()
    zr = np.einsum("nab,nbr->nar", Minv, x)
    assert np.max(np.abs(z - zr)) <= 1e-12 * np.max(np.abs(zr))


@pytest.fixture(scope="module")
def curved_crust(gpu_lib):
    m = meshgen.curve_edges(meshgen.crust_mesh(12, 12, 6), meshgen.rng_for(85, 0), amp=0.08)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(85, 1), nrhs=16)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    print(f"[curved crust 12x12x6] DOF={m.n_dof}: oracle sparse LU", flush=True)
    return m, ebe.Mesh.from_generated(m, curved=True), f, solve.sparse_solve(K, f, m.fixed)


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precond,mode,tol,bound", [(ebe.PREC_MG3, ebe.MODE_MIXED, 1e-8, 1e-6),
                                                    (ebe.PREC_MG2, ebe.MODE_MIXED, 1e-8, 1e-6),
                                                    (ebe.PREC_MG3, ebe.MODE_FP64, 1e-13, 1e-10)])
def test_curved_crust_solves_match_direct_solution(curved_crust, precond, mode, tol, bound):
    m, gm, f, ud = curved_crust
    u, st = gm.solve(to_dev(f, np.float64), precond=precond, mode=mode, tol=tol)
    print(f"[curved crust precond={precond} mode={mode}] {st}", flush=True)
    assert st["status"] == ebe.OK and st["precond_used"] == precond
    assert rel_err(u.cpu().numpy(), ud) <= bound


def test_curved_mesh_refusals(curved):
    m, gm, K, absK, kap = curved
    u = to_dev(np.zeros((m.n_nodes, 3, 2)), np.float64)
    with pytest.raises(ebe.EbeError) as ei:
        gm.adjoint_grad(u, u)
    assert ei.value.status == ebe.ERR_ARG and "curved" in str(ei.value)
    try:  # a form the curved kernel does not come in is kept as a preference; the gather form runs
        for form in (ebe.FORM_STAGED, ebe.FORM_PIPELINED, ebe.FORM_COLOURED, ebe.FORM_DETERMINISTIC):
            gm.set_form(0, torch.float32, 4, form)
            assert gm.form(0, torch.float32, 4) == ebe.FORM_GATHER
    finally:
        gm.set_form(0, torch.float32, 4, ebe.FORM_AUTO)
    sides = np.zeros(m.n_elem, dtype=np.int8)
    sides[0] = 1
    with pytest.raises(ebe.EbeError) as ei:
        ebe.Fault(gm, sides, np.array([m.conn[0, 0]], dtype=np.int32), np.ones((1, 1)), np.array([[1.0, 0, 0]]))
    assert ei.value.status == ebe.ERR_ARG and "curved" in str(ei.value)
    with pytest.raises(ebe.EbeError) as ei:  # the curved kernel sums with LDS atomics
        gm.solve(to_dev(np.zeros((m.n_nodes, 3, 2)), np.float64), deterministic=1)
    assert ei.value.status == ebe.ERR_ARG
    ms = gm.autotune(0, torch.float32, 4)
    assert ms[ebe.FORM_GATHER] > 0 and all(ms[f] < 0 for f in (ebe.FORM_STAGED, ebe.FORM_PIPELINED,
                                                                 ebe.FORM_COLOURED, ebe.FORM_DETERMINISTIC))


def test_full_size_curved_matvec_sampled(gpu_lib):
    """The 64^3 x 6 cube mapped by x -> x + 0.25 x^2 (bench.py's curved
    workload), FP32 with 16 cases: every node of the first and last element
    ranges and a random sample, against the oracle's element products around
    them."""
    from tests.helpers import restricted_matvec
    m = meshgen.quadratic_map(meshgen.matvec_mesh(64), 0.25)
    gm = ebe.Mesh.from_generated(m, curved=True)
    rng = meshgen.rng_for(86, 0)
    x = meshgen.random_vectors(rng, m.n_nodes, 16).astype(np.float32).astype(np.float64)
    y = gm.matvec(to_dev(x, np.float32)).cpu().numpy().astype(np.float64)
    nodes = np.unique(np.concatenate([m.conn[:96].ravel(), m.conn[-96:].ravel(),
                                      rng.choice(m.n_nodes, 256, replace=False)]))
    ref, absKx = restricted_matvec(m, x, nodes)
    touched = np.nonzero(np.isin(m.conn, nodes).any(axis=1))[0]
    sub = meshgen.Mesh(xyz=m.xyz, conn=m.conn[touched], n_vertices=m.n_vertices, young=m.young[touched],
                       poisson=m.poisson[touched], fixed=m.fixed)
    tol = C_TOL[np.float32] * kappa_points(sub) * unit_roundoff(np.float32) * absKx + 1e-300
    worst = float(np.max(np.abs(y[nodes] - ref) / tol))
    print(f"[curved 64^3 f32 n=16] {nodes.size} nodes, worst err / bound {worst:.3g}", flush=True)
    assert worst <= 1.0


def test_batch_with_a_curved_mesh_is_never_merged(gpu_lib):
    """A batch of small meshes with merging on: the straight ones form a
    merged group, the curved one is solved on its own with its own
    (curved) operator; every result matches the oracle's direct solve."""
    ms = [meshgen.crust_mesh(3, 3, 2), meshgen.crust_mesh(4, 3, 2),
          meshgen.curve_edges(meshgen.crust_mesh(4, 4, 2), meshgen.rng_for(87, 0), amp=0.06)]
    gms, fs, refs = [], [], []
    for k, m in enumerate(ms):
        f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(87, 10 + k), nrhs=9)
        K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
        gms.append(ebe.Mesh.from_generated(m, curved=(k == 2)))
        fs.append(to_dev(f, np.float64))
        refs.append(solve.sparse_solve(K, f, m.fixed))
    info = {}
    us, sts = ebe.batch_solve(gms, fs, tol=1e-9, info=info, merge_elems=150000)
    print(f"[batch with a curved mesh] {info}", flush=True)
    assert info["group_of"][2] == -1 and info["group_of"][0] == info["group_of"][1] >= 0
    for u, r, st in zip(us, refs, sts):
        assert st["status"] == ebe.OK and st["max_rel_res"] <= 1e-9
        assert rel_err(u.cpu().numpy(), r) <= 1e-6
