"""GPU solves (Algorithm 1 and PCGE) against the oracle's direct solutions,
plus the adjoint gradient through torch.autograd."""
import copy

import numpy as np
import pytest
import torch

from oracle import adjoint, fem, solve
from paper_1710_08679_amd import ebe, meshgen
from paper_1710_08679_amd.autograd import surface_misfit

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def cube(gpu_lib):
    m = meshgen.cube_mesh(4)
    f = meshgen.top_face_random_loads(m, meshgen.rng_for(1, 0), nrhs=1)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    return m, ebe.Mesh.from_generated(m), f, K, solve.dense_solve(K, f, m.fixed)


def test_small_cube_pcge_fp64_reaches_dense_solution(cube):
    m, gm, f, K, ud = cube
    print("[cube 4^3] PCGE FP64 tol 1e-10", flush=True)
    u, st = gm.solve(dev(f), precond=ebe.PREC_PCGE, mode=ebe.MODE_FP64, tol=1e-10)
    assert st["status"] == ebe.OK and st["max_rel_res"] <= 1e-10
    un = u.cpu().numpy()
    r = solve.residual(K, un, f, m.fixed)
    assert np.linalg.norm(r) <= 1.5e-10 * np.linalg.norm(f)  # oracle residual of the GPU answer
    u2, st2 = gm.solve(dev(f), precond=ebe.PREC_PCGE, mode=ebe.MODE_FP64, tol=1e-13)
    assert rel_err(u2.cpu().numpy(), ud) <= 1e-10


@pytest.mark.parametrize("precond,mode", [(ebe.PREC_MG2, ebe.MODE_MIXED), (ebe.PREC_MG2, ebe.MODE_FP64),
                                          (ebe.PREC_MG3, ebe.MODE_MIXED), (ebe.PREC_MG3, ebe.MODE_FP64)])
def test_small_cube_mg2(cube, precond, mode):
    m, gm, f, K, ud = cube
    u, st = gm.solve(dev(f), precond=precond, mode=mode, tol=1e-12)
    assert st["status"] == ebe.OK
    assert rel_err(u.cpu().numpy(), ud) <= 1e-10


@pytest.fixture(scope="module")
def crust(gpu_lib):
    m = meshgen.crust_mesh(12, 12, 6)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(3, 2), nrhs=16)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    print(f"[crust 12x12x6] DOF={m.n_dof}: oracle sparse LU", flush=True)
    return m, ebe.Mesh.from_generated(m), f, K, solve.sparse_solve(K, f, m.fixed)


@pytest.mark.parametrize("form", [ebe.FORM_GATHER, ebe.FORM_STAGED, ebe.FORM_PIPELINED, ebe.FORM_ASSEMBLED,
                                  ebe.FORM_COLOURED, ebe.FORM_DETERMINISTIC])
def test_crust_mixed_mg2_in_each_product_form(crust, form):
    """Every product of the solve (outer FP64, inner FP32 on both levels,
    each also forming (p, K p)) in one given form (the assembled form exists
    at the linear level only, the coloured form at the quadratic level only:
    elsewhere the gather form runs)."""
    m, gm, f, K, ud = crust
    keys = [(0, torch.float64), (0, torch.float32), (1, torch.float32)]
    try:
        for level, dt in keys:
            only = (form == ebe.FORM_ASSEMBLED and level == 0) or (
                form in (ebe.FORM_COLOURED, ebe.FORM_DETERMINISTIC) and level == 1)
            gm.set_form(level, dt, 16, ebe.FORM_GATHER if only else form)
        u, st = gm.solve(dev(f), precond=ebe.PREC_MG2, mode=ebe.MODE_MIXED, tol=1e-8)
    finally:
        for level, dt in keys:
            gm.set_form(level, dt, 16, ebe.FORM_AUTO)
    print(f"[crust mixed MG2 form={form}] {st}", flush=True)
    assert st["status"] == ebe.OK and st["max_rel_res"] <= 1e-8
    assert rel_err(u.cpu().numpy(), ud) <= 1e-6


@pytest.mark.parametrize("precond,mode,tol,bound", [(ebe.PREC_MG3, ebe.MODE_MIXED, 1e-8, 1e-6),
                                                    (ebe.PREC_MG2, ebe.MODE_FP64, 1e-13, 1e-10),
                                                    (ebe.PREC_PCGE, ebe.MODE_FP64, 1e-11, 1e-8)])
def test_deterministic_solves_are_bitwise_reproducible(crust, precond, mode, tol, bound):
    """opts.deterministic: two solves (the second on a side stream, with graph
    capture) give the same bits and the same statistics, and the solution
    matches the oracle's direct solve."""
    m, gm, f, K, ud = crust
    fd = dev(f)
    u1, st1 = gm.solve(fd, precond=precond, mode=mode, tol=tol, deterministic=1)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        u2, st2 = gm.solve(fd, precond=precond, mode=mode, tol=tol, deterministic=1, stream=side)
    side.synchronize()
    print(f"[deterministic precond={precond} mode={mode}] {st1} / {st2}", flush=True)
    assert st1["status"] == ebe.OK and torch.equal(u1, u2)
    for k in ("outer_iters", "inner_iters", "max_rel_res"):
        assert st1[k] == st2[k], k
    assert rel_err(u1.cpu().numpy(), ud) <= bound


@pytest.mark.parametrize("coarse_guess", [0, 1])
def test_crust_mixed_mg2_within_1e6(crust, coarse_guess):
    m, gm, f, K, ud = crust
    u, st = gm.solve(dev(f), precond=ebe.PREC_MG2, mode=ebe.MODE_MIXED, tol=1e-8, coarse_guess=coarse_guess)
    print(f"[crust mixed MG2] {st}", flush=True)
    assert st["status"] == ebe.OK
    un = u.cpu().numpy()
    for j in range(f.shape[2]):
        assert rel_err(un[:, :, j], ud[:, :, j]) <= 1e-6
    assert np.all(un[m.fixed.astype(bool)] == 0)


def test_crust_fp64_paths_within_1e10(crust):
    m, gm, f, K, ud = crust
    for precond in (ebe.PREC_PCGE, ebe.PREC_MG2, ebe.PREC_MG3):
        u, st = gm.solve(dev(f), precond=precond, mode=ebe.MODE_FP64, tol=1e-13)
        print(f"[crust FP64 precond={precond}] {st}", flush=True)
        assert st["status"] == ebe.OK
        assert rel_err(u.cpu().numpy(), ud) <= 1e-10


def test_multi_case_equals_single_cases_and_zero_case(crust):
    m, gm, f, K, ud = crust
    f4 = f[:, :, :4].copy()
    f4[:, :, 2] = 0.0
    u, st = gm.solve(dev(f4), tol=1e-9)
    assert st["status"] == ebe.OK
    un = u.cpu().numpy()
    assert np.all(un[:, :, 2] == 0.0)
    for j in (0, 3):
        uj, _ = gm.solve(dev(f4[:, :, j:j + 1]), tol=1e-9)
        assert rel_err(un[:, :, j], uj.cpu().numpy()[:, :, 0]) <= 1e-7


def test_initial_guess_and_iteration_cap(crust):
    m, gm, f, K, ud = crust
    u0 = dev(ud[:, :, :2])
    u, st = gm.solve(dev(f[:, :, :2]), u=u0, use_x0=1, precond=ebe.PREC_PCGE, mode=ebe.MODE_FP64, tol=1e-8)
    assert st["status"] == ebe.OK and st["outer_iters"] == 0
    u, st = gm.solve(dev(f[:, :, :2]), precond=ebe.PREC_PCGE, mode=ebe.MODE_FP64, tol=1e-12, max_outer=3)
    assert st["status"] == ebe.NOT_CONVERGED and st["outer_iters"] == 3


@pytest.mark.parametrize("precond,mode", [(ebe.PREC_MG2, ebe.MODE_MIXED), (ebe.PREC_PCGE, ebe.MODE_FP64)])
def test_graph_replays_match_eager_solves(crust, precond, mode):
    """On a non-default stream the fixed runs of steps between convergence
    checks are captured once and replayed.  Three solves into the same output
    (replaying the same graphs), with eager work and host synchronisation in
    between, each reach the eager solve's answer."""
    m, gm, f, K, ud = crust
    fd = dev(f[:, :, :5])
    ref = ud[:, :, :5]
    s = torch.cuda.Stream()
    opts_e = ebe.default_opts(precond=precond, mode=mode, tol=1e-9, graphs=0)
    opts_g = ebe.default_opts(precond=precond, mode=mode, tol=1e-9, graphs=1)
    with torch.cuda.stream(s):
        ue, ste = gm.solve(fd, opts=opts_e, stream=s)
        ug = torch.empty_like(fd)
        for rep in range(3):
            ug.fill_(float(rep + 1))  # eager work between replays
            _, stg = gm.solve(fd, u=ug, opts=opts_g, stream=s)
            s.synchronize()
            print(f"[graphs precond={precond} rep={rep}] {stg} (eager {ste})", flush=True)
            assert stg["status"] == ebe.OK and stg["max_rel_res"] <= 1e-9
            assert abs(stg["outer_iters"] - ste["outer_iters"]) <= 1
            assert float((ug - ue).norm() / ue.norm()) <= 1e-6
            assert rel_err(ug.cpu().numpy(), ref) <= 1e-6


def test_graph_capture_follows_product_form(crust):
    """Graphs are keyed by the product forms as well as by buffers: after the
    form of a product changes, the next solve on a stream captures new graphs
    instead of replaying ones whose kernels were picked for the old form."""
    m, gm, f, K, ud = crust
    fd = dev(f[:, :, :4])
    ref = ud[:, :, :4]
    keys = [(0, torch.float64), (0, torch.float32), (1, torch.float32)]
    s = torch.cuda.Stream()
    opts = ebe.default_opts(precond=ebe.PREC_MG2, mode=ebe.MODE_MIXED, tol=1e-8, graphs=1)
    try:
        with torch.cuda.stream(s):
            for form, fresh in ((ebe.FORM_GATHER, True), (ebe.FORM_GATHER, False), (ebe.FORM_PIPELINED, True),
                                (ebe.FORM_GATHER, False)):
                for level, dt in keys:
                    gm.set_form(level, dt, 4, form)
                u, st = gm.solve(fd, opts=opts, stream=s)
                s.synchronize()
                print(f"[graph keys form={form}] {st}", flush=True)
                assert st["status"] == ebe.OK
                assert (st["graphs_captured"] > 0) == fresh, st
                assert rel_err(u.cpu().numpy(), ref) <= 1e-6
    finally:
        for level, dt in keys:
            gm.set_form(level, dt, 4, ebe.FORM_AUTO)


def test_mg3_falls_back_to_mg2_on_long_coarse_rows(gpu_lib):
    """A hub corner shared by 850 two-element arms makes every level-2 row
    couple 850 aggregates, past what the level-2 set-up can sum: a solve asked
    for MG3 runs MG2, reports it, and still reaches the direct solution."""
    m = meshgen.hub_mesh(850)
    gm = ebe.Mesh.from_generated(m)
    f = meshgen.random_vectors(meshgen.rng_for(9, 1), m.n_nodes, 3)
    f[m.fixed.astype(bool)] = 0.0
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    ud = solve.sparse_solve(K, f, m.fixed)
    u, st = gm.solve(dev(f), precond=ebe.PREC_MG3, tol=1e-9)
    print(f"[hub mesh, MG3 asked] {st}", flush=True)
    assert st["status"] == ebe.OK and st["precond_used"] == ebe.PREC_MG2
    assert rel_err(u.cpu().numpy(), ud) <= 1e-6
    u, st = gm.solve(dev(f), precond=ebe.PREC_PCGE, mode=ebe.MODE_FP64, tol=1e-9)
    assert st["status"] == ebe.OK and st["precond_used"] == ebe.PREC_PCGE


@pytest.mark.parametrize("precond,mode,tol,bound", [(ebe.PREC_MG3, ebe.MODE_MIXED, 1e-8, 1e-6),
                                                    (ebe.PREC_MG3, ebe.MODE_FP64, 1e-13, 1e-10),
                                                    (ebe.PREC_MG2, ebe.MODE_MIXED, 1e-8, 1e-6)])
def test_shuffled_mesh_solves(gpu_lib, precond, mode, tol, bound):
    """Algorithm 1 on a mesh with shuffled elements and node ids: patches cut
    by the node limit on every level, aggregates of an unordered corner graph."""
    m = meshgen.shuffled(meshgen.crust_mesh(10, 10, 5, jitter=0.2), meshgen.rng_for(3, 77))
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(3, 78), nrhs=5)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    ud = solve.sparse_solve(K, f, m.fixed)
    gm = ebe.Mesh.from_generated(m)
    u, st = gm.solve(dev(f), precond=precond, mode=mode, tol=tol)
    print(f"[shuffled crust precond={precond} mode={mode}] {st}", flush=True)
    assert st["status"] == ebe.OK and st["precond_used"] == precond
    assert rel_err(u.cpu().numpy(), ud) <= bound


def test_full_size_crust_mixed_solve(gpu_lib):
    """The 96x96x48 crust workload (10.8M DOF, 16 cases) as bench.py solves it:
    the FP64 residual of the mixed solution meets the tolerance, and that
    residual agrees with the oracle's element products at sampled nodes."""
    from tests.helpers import kappa_max, sampled_matvec, tol_factor
    m = meshgen.crust_mesh(96, 96, 48)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(3, 2), nrhs=16)
    gm = ebe.Mesh.from_generated(m)
    fd = dev(f)
    print(f"[crust 96x96x48] DOF={m.n_dof}", flush=True)
    u, st = gm.solve(fd, precond=ebe.PREC_MG3, mode=ebe.MODE_MIXED, tol=1e-8)
    print(f"[crust 96x96x48 mixed MG3] {st}", flush=True)
    assert st["status"] == ebe.OK and st["max_rel_res"] <= 1e-8
    fixed = torch.from_numpy(m.fixed.astype(bool)).cuda()
    fb = fd.clone()
    fb[fixed] = 0
    r = fb - gm.matvec(u, apply_bc=True)
    rel = (torch.linalg.vector_norm(r.reshape(-1, 16), dim=0) / torch.linalg.vector_norm(fb.reshape(-1, 16), dim=0))
    assert float(rel.max()) <= 2e-8, rel
    # oracle K u at sampled free nodes (and the nodes carrying the loads)
    free = np.nonzero(~m.fixed.astype(bool).any(axis=1))[0]
    loaded = np.unique(np.nonzero(np.abs(f).sum(axis=(1, 2)))[0])
    nodes = np.concatenate([meshgen.rng_for(3, 90).choice(free, size=48, replace=False), loaded[:16]])
    un = u.cpu().numpy()
    ref, bnd = sampled_matvec(m, un, nodes)
    Ku = gm.matvec(u).cpu().numpy()[nodes]
    tol = tol_factor(np.float64, kappa_max(m)) * bnd
    assert np.all(np.abs(Ku - ref) <= tol), float(np.max(np.abs(Ku - ref) / tol))


def test_nonfinite_input_is_reported(crust):
    m, gm, f, K, ud = crust
    fb = f[:, :, :1].copy()
    fb[np.nonzero(~m.fixed.astype(bool).any(axis=1))[0][0], 0, 0] = np.nan
    with pytest.raises(ebe.EbeError) as ei:
        gm.solve(dev(fb))
    assert ei.value.status == ebe.ERR_NONFINITE


@pytest.mark.parametrize("precond", [ebe.PREC_MG2, ebe.PREC_MG3])
def test_crust_mixed_with_fp16_coarse_operators(crust, precond):
    """Low-precision preconditioner experiment: the linear level's K1 and the
    level-2 A2 stored in FP16 (FP32 arithmetic).  The FP64 outer loop still
    reaches the tolerance and the direct solution; the iteration counts of
    both settings are printed for comparison."""
    m, gm, f, K, ud = crust
    u0, st0 = gm.solve(dev(f), precond=precond, mode=ebe.MODE_MIXED, tol=1e-8)
    u, st = gm.solve(dev(f), precond=precond, mode=ebe.MODE_MIXED, tol=1e-8, coarse_half=1)
    print(f"[fp16 coarse precond={precond}] FP32 coarse {st0['outer_iters']} {st0['inner_iters']}, "
          f"FP16 coarse {st['outer_iters']} {st['inner_iters']}", flush=True)
    assert st["status"] == ebe.OK and st["max_rel_res"] <= 1e-8
    assert rel_err(u.cpu().numpy(), ud) <= 1e-6
    assert st["outer_iters"] <= 2 * st0["outer_iters"]


def test_batch_of_uneven_meshes(gpu_lib):
    ms, gms, fs, refs = [], [], [], []
    for k, (g, n) in enumerate([((4, 4, 2), 3), ((6, 6, 3), 1), ((5, 5, 3), 16)]):
        m = meshgen.crust_mesh(*g)
        f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(5, k), nrhs=n)
        K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
        ms.append(m)
        gms.append(ebe.Mesh.from_generated(m))
        fs.append(dev(f))
        refs.append(solve.sparse_solve(K, f, m.fixed))
    us, sts = ebe.batch_solve(gms, fs, tol=1e-8)
    for u, r, st in zip(us, refs, sts):
        assert st["status"] == ebe.OK
        assert rel_err(u.cpu().numpy(), r) <= 1e-6


def test_batch_with_more_meshes_than_lanes_and_an_error(gpu_lib):
    """Seven meshes over the batch's worker streams: each result equals that
    mesh's own solve; a non-finite right-hand side fails with its mesh named."""
    grids = [(3, 3, 2), (4, 3, 2), (4, 4, 2), (5, 4, 3), (3, 5, 2), (6, 5, 3), (4, 4, 4)]
    gms, fs = [], []
    for k, g in enumerate(grids):
        m = meshgen.crust_mesh(*g)
        f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(5, 20 + k), nrhs=1 + (5 * k) % 16)
        gms.append(ebe.Mesh.from_generated(m))
        fs.append(dev(f))
    opts = ebe.default_opts(tol=1e-10)
    us, sts = ebe.batch_solve(gms, fs, opts=opts)
    for gm, f, u, st in zip(gms, fs, us, sts):
        assert st["status"] == ebe.OK and st["max_rel_res"] <= 1e-10
        u1, st1 = gm.solve(f, opts=opts)
        assert st1["status"] == ebe.OK
        assert float((u - u1).norm() / u1.norm()) <= 1e-6
    bad = [f.clone() for f in fs]
    free = int(np.nonzero(~meshgen.crust_mesh(*grids[4]).fixed.astype(bool).any(axis=1))[0][0])
    bad[4][free, 1, 0] = float("nan")
    with pytest.raises(ebe.EbeError) as ei:
        ebe.batch_solve(gms, bad, opts=opts)
    assert ei.value.status == ebe.ERR_NONFINITE
    assert "mesh 4" in str(ei.value)


def test_batch_merges_small_meshes(gpu_lib):
    """Meshes with 9-16 cases are solved as one merged block-diagonal system
    (one launch per step over all their patches); a mesh with 2 cases alone.
    Each result matches the oracle's direct solve, each member's reported
    residual is its own (recomputed with its operator), and merging off
    gives the same solutions."""
    grids = [(3, 3, 2), (4, 3, 2), (4, 4, 2), (5, 4, 3), (3, 5, 2)]
    nrhs = [12, 9, 16, 10, 2]
    gms, fs, refs = [], [], []
    for k, (g, n) in enumerate(zip(grids, nrhs)):
        m = meshgen.crust_mesh(*g)
        f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(5, 40 + k), nrhs=n)
        f[:, :, -1] *= 1e3 ** (k % 3)  # cases of very different size share the merged system
        K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
        gms.append(ebe.Mesh.from_generated(m))
        fs.append(dev(f))
        refs.append(solve.sparse_solve(K, f, m.fixed))
    info = {}
    us, sts = ebe.batch_solve(gms, fs, tol=1e-9, info=info, merge_elems=150000)
    print(f"[merged batch] {info}, merged {[s['merged'] for s in sts]}", flush=True)
    assert info["groups"] == 1 and info["group_of"] == [0, 0, 0, 0, -1]
    assert [s["merged"] for s in sts] == [4, 4, 4, 4, 0]
    for u, r, st in zip(us, refs, sts):
        assert st["status"] == ebe.OK and st["max_rel_res"] <= 1e-9
        assert rel_err(u.cpu().numpy(), r) <= 1e-6
    info0 = {}
    us0, sts0 = ebe.batch_solve(gms, fs, tol=1e-9, merge_elems=0, info=info0)
    assert info0["groups"] == 0 and all(s["merged"] == 0 for s in sts0)
    for u, u0 in zip(us, us0):
        assert float((u - u0).norm() / u0.norm()) <= 1e-6


# ---------------------------------------------------------------------------
# adjoint gradient
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def adj(gpu_lib):
    m = meshgen.adjoint_mesh(8, 8, 4)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(4, 3), nrhs=4)
    S = meshgen.top_surface_dofs(m)
    d = 1e-3 * meshgen.rng_for(4, 4).standard_normal((S.size, 4))
    L, g, u, lam = adjoint.gradient(m.xyz, m.conn, m.young, m.poisson, m.fixed, f, S, d)
    return m, ebe.Mesh.from_generated(m), f, S, d, L, g


@pytest.mark.parametrize("grad_dtype,tol", [(torch.float64, 1e-8), (torch.float32, 1e-4)])
def test_autograd_gradient_matches_oracle(adj, grad_dtype, tol):
    m, gm, f, S, d, L, g = adj
    E = dev(m.young).requires_grad_(True)
    opts = ebe.default_opts(precond=ebe.PREC_MG2, mode=ebe.MODE_MIXED, tol=1e-12)
    loss = surface_misfit(E, gm, dev(m.poisson), dev(f), torch.from_numpy(S).cuda(), dev(d), opts, grad_dtype)
    loss.backward()
    assert abs(float(loss) - L) <= 1e-9 * abs(L)
    gg = E.grad.cpu().numpy()
    assert np.max(np.abs(gg - g)) <= tol * np.max(np.abs(g))


def test_gradient_central_differences_on_gpu(adj):
    m, gm, f, S, d, L, g = adj
    opts = ebe.default_opts(precond=ebe.PREC_PCGE, mode=ebe.MODE_FP64, tol=1e-13)
    Sd = torch.from_numpy(S).cuda()
    E = dev(m.young).requires_grad_(True)
    loss = surface_misfit(E, gm, dev(m.poisson), dev(f), Sd, dev(d), opts)
    loss.backward()
    gg = E.grad.cpu().numpy()
    for e in meshgen.rng_for(4, 5).choice(m.n_elem, size=20, replace=False):
        h = 1e-4 * m.young[e]
        vals = []
        for sgn in (1, -1):
            Ep = m.young.copy()
            Ep[e] += sgn * h
            with torch.no_grad():
                vals.append(float(surface_misfit(dev(Ep), gm, dev(m.poisson), dev(f), Sd, dev(d), opts)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gg[e]) <= 1e-5 * np.max(np.abs(gg))


def test_adjoint_workload_central_differences(gpu_lib):
    """The adjoint workload at its stated size (64x64x32 hexes x 6 = 786,432
    tets, 4 cases, lognormal moduli, top-surface misfit): dL/dE from the FP64
    and the FP32 element-gradient kernels against central differences of L
    on 20 seeded elements, every solve FP64 to 1e-13."""
    m = meshgen.adjoint_mesh(64, 64, 32)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(4, 3), nrhs=4)
    S = meshgen.top_surface_dofs(m)
    gm = ebe.Mesh.from_generated(m)
    print(f"[adjoint workload] E={m.n_elem} DOF={m.n_dof}", flush=True)
    opts = ebe.default_opts(precond=ebe.PREC_MG3, mode=ebe.MODE_FP64, tol=1e-13)
    Sd = torch.from_numpy(S).cuda()
    # targets: the unperturbed layered model's surface response plus 1% noise
    base = copy.copy(m)
    meshgen.set_layers_sinusoidal(base, meshgen.rng_for(4, 1))  # rebinds base.young / base.poisson only
    assert np.array_equal(base.poisson, m.poisson) and not np.array_equal(base.young, m.young)
    gm.set_material(dev(base.young), dev(base.poisson))
    u0, _ = gm.solve(dev(f), opts=opts)
    s0 = u0.view(-1, 4)[Sd]
    d = s0 + 0.01 * float(s0.abs().mean()) * dev(meshgen.rng_for(4, 4).standard_normal((S.size, 4)))
    grads = {}
    for gdt in (torch.float64, torch.float32):
        E = dev(m.young).requires_grad_(True)
        loss = surface_misfit(E, gm, dev(m.poisson), dev(f), Sd, d, opts, gdt)
        loss.backward()
        grads[gdt] = E.grad.cpu().numpy()
    g64, g32 = grads[torch.float64], grads[torch.float32]
    scale = float(np.max(np.abs(g64)))
    assert np.max(np.abs(g32 - g64)) <= 1e-4 * scale
    for k, e in enumerate(meshgen.rng_for(4, 5).choice(m.n_elem, size=20, replace=False)):
        h = 1e-4 * m.young[e]
        vals = []
        for sgn in (1, -1):
            Ep = m.young.copy()
            Ep[e] += sgn * h
            with torch.no_grad():
                vals.append(float(surface_misfit(dev(Ep), gm, dev(m.poisson), dev(f), Sd, d, opts)))
        fd = (vals[0] - vals[1]) / (2 * h)
        print(f"[adjoint fd {k}] e={e} fd={fd:.6e} g64={g64[e]:.6e} g32={g32[e]:.6e}", flush=True)
        assert abs(fd - g64[e]) <= 1e-5 * scale
        assert abs(fd - g32[e]) <= 1e-5 * scale
