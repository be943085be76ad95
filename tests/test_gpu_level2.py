"""GPU parity of level 2 (smoothed aggregation of the corner mesh) against the
oracle, through the C ABI: the aggregates (bit-exact), P2 and P2^T, A2 x, the
level-2 block Jacobi, and three-level solves against the direct solution.
Bounds are relative to the absolute values of the terms summed (|P2|+ |x|
with |P2|+ = |T| + omega |D1^-1| |K1p| |T|, and |P2|+^T |K1p| |P2|+ |x|), which
bound the rounding of the sums whatever their order."""
import scipy.sparse as sp
import numpy as np
import pytest
import torch

from oracle import alg1, amg, fem, solve
from paper_1710_08679_amd import ebe, meshgen
from tests.helpers import parity_mesh

pytestmark = pytest.mark.gpu

DT = {np.float64: torch.float64, np.float32: torch.float32}


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def dof_apply(P, v):
    M, _, n = v.shape
    return (P @ v.reshape(3 * M, n)).reshape(P.shape[0] // 3, 3, n)


@pytest.fixture(scope="module")
def lv2(gpu_lib):
    m = parity_mesh(9, 7, 5, seed=3, bc=True)
    K1 = fem.assemble(m.xyz, m.conn, m.young, m.poisson, order=1, n_nodes=m.n_vertices)
    agg, na, P2, A2, cfx = amg.level2(m.conn, m.n_vertices, K1, m.fixed)
    T = amg.prolongation_p2(agg, na, m.fixed)
    K1p = abs(amg.projected(K1, m.fixed))
    D = sp.block_diag(list(np.abs(solve.block_jacobi_inverse(K1, m.fixed[:m.n_vertices], m.n_vertices)))).tocsr()
    absP = (abs(T) + amg.OMEGA * (D @ (K1p @ abs(T)))).tocsr()
    absA = (absP.T @ K1p @ absP).tocsr()
    print(f"[level 2] Nv={m.n_vertices} aggregates={na}", flush=True)
    return m, ebe.Mesh.from_generated(m), agg, na, P2, A2, cfx, (absP, absA)


def test_aggregates_equal_the_oracle(lv2):
    m, gm, agg, na, *_ = lv2
    n, a = gm.level2_info()
    assert n == na and np.array_equal(a, agg)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [5, 8, 16])
def test_transfers_match_oracle(lv2, dtype, nrhs):
    m, gm, agg, na, P2, A2, cfx, (absP, absA) = lv2
    rng = meshgen.rng_for(93, nrhs)
    x2 = rng.standard_normal((na, 3, nrhs)).astype(dtype)
    x1 = rng.standard_normal((m.n_vertices, 3, nrhs)).astype(dtype)
    y1 = gm.prolong_l2(to_dev(x2, dtype)).cpu().numpy().astype(np.float64)
    y2 = gm.restrict_l2(to_dev(x1, dtype)).cpu().numpy().astype(np.float64)
    r1 = dof_apply(P2, x2.astype(np.float64))
    r2 = dof_apply(P2.T.tocsr(), x1.astype(np.float64))
    r2[cfx] = 0
    b1 = dof_apply(absP, np.abs(x2.astype(np.float64))) + 1e-300
    b2 = dof_apply(absP.T.tocsr(), np.abs(x1.astype(np.float64))) + 1e-300
    c = 1e-13 if dtype == np.float64 else 8 * float(np.finfo(np.float32).eps)
    assert np.max(np.abs(y1 - r1) / b1) <= c
    assert np.max(np.abs(y2 - r2) / b2) <= c
    assert np.all(y2[cfx] == 0)
    assert np.all(y1[m.fixed[:m.n_vertices].astype(bool)] == 0)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("nrhs", [1, 4, 7, 16])
def test_a2_product_matches_oracle(lv2, dtype, nrhs):
    m, gm, agg, na, P2, A2, cfx, (absP, absA) = lv2
    x = meshgen.rng_for(94, nrhs).standard_normal((na, 3, nrhs)).astype(dtype)
    xd = x.astype(np.float64)
    y = gm.matvec_l2(to_dev(x, dtype)).cpu().numpy().astype(np.float64)
    yb = gm.matvec_l2(to_dev(x, dtype), apply_bc=True).cpu().numpy().astype(np.float64)
    ref = dof_apply(A2, xd)
    xm = xd.copy()
    xm[cfx] = 0
    refb = dof_apply(A2, xm)
    refb[cfx] = 0
    # |P2|+^T |K1p| |P2|+ |x| bounds the rounding of the (summed, then
    # rounded) blocks and of the products
    bound = dof_apply(absA, np.abs(xd)) + 1e-300
    c = 1e-12 if dtype == np.float64 else 64 * float(np.finfo(np.float32).eps)
    assert np.max(np.abs(y - ref) / bound) <= c
    assert np.max(np.abs(yb - refb) / bound) <= c
    assert np.all(yb[cfx] == 0)


def test_level2_blocks_match_oracle(lv2):
    """Diagonal blocks of A2 elementwise within the rounding bound of their
    sums: an entry of A2 = P2^T K1p P2 is a sum of k products, each factor
    itself a rounded sum (K1 of element blocks, P2 = T - omega D1^-1 K1p T
    with the inverted 3x3 blocks D1^-1), so |error| <= (k + 16 kappa_D) u
    times the same sums of absolute terms, with the element blocks' absolute
    values in place of |K1| (cancellation inside K1 is not free), k the
    largest term count of a diagonal-block entry and kappa_D the largest
    condition number of the blocks D1."""
    m, gm, agg, na, P2, A2, cfx, _ = lv2
    got = gm.diag_blocks(2).cpu().numpy()
    ref = fem.diag_blocks(A2, na)
    nv = m.n_vertices
    Ke = np.abs(fem.element_stiffness_p1(m.xyz[m.conn[:, :4]], m.young, m.poisson))
    dm = (3 * m.conn[:, :4, None].astype(np.int64) + np.arange(3)).reshape(m.n_elem, 12)
    absK1 = sp.coo_matrix((Ke.ravel(), (np.repeat(dm, 12, axis=1).ravel(), np.tile(dm, (1, 12)).ravel())),
                          shape=(3 * nv, 3 * nv)).tocsr()
    absK1p = amg.projected(absK1, m.fixed)
    K1 = fem.assemble(m.xyz, m.conn, m.young, m.poisson, order=1, n_nodes=nv)
    Dblk = fem.diag_blocks(amg.projected(K1, m.fixed), nv)
    Dinv = solve.block_jacobi_inverse(K1, m.fixed[:nv], nv)
    free = ~m.fixed[:nv].astype(bool)
    kap = max(np.linalg.cond(Dblk[v][np.ix_(free[v], free[v])]) for v in range(nv) if free[v].any())
    T = amg.prolongation_p2(agg, na, m.fixed)
    absP = (abs(T) + amg.OMEGA * (sp.block_diag(list(np.abs(Dinv))).tocsr() @ (absK1p @ abs(T)))).tocsr()
    bound = fem.diag_blocks((absP.T @ absK1p @ absP).tocsr(), na)
    pat = lambda a: (abs(a) > 0).astype(np.float64)  # noqa: E731
    k = fem.diag_blocks((pat(absP).T @ pat(absK1p) @ pat(absP)).tocsr(), na).max()
    u = np.finfo(np.float64).eps / 2
    tol = (k + 16 * kap) * u * bound + 1e-300
    worst = float(np.max(np.abs(got - ref) / tol))
    print(f"[level-2 blocks] k={k:.0f} kappa_D={kap:.3g}, worst err / bound {worst:.3g}", flush=True)
    assert worst <= 1.0
    Minv = solve.block_jacobi_inverse(A2, cfx, na)
    x = meshgen.rng_for(95, 0).standard_normal((na, 3, 4))
    x[cfx] = 0.0
    z = gm.block_jacobi(to_dev(x, np.float64), level=2).cpu().numpy()
    zr = np.einsum("nab,nbr->nar", Minv, x)
    assert np.max(np.abs(z - zr)) <= 1e-12 * np.max(np.abs(zr))


def test_level2_follows_a_material_change(lv2):
    m, gm, agg, na, P2, A2, cfx, (absP, absA) = lv2
    E2 = m.young * 1.7
    gm.set_material(to_dev(E2, np.float64), to_dev(m.poisson, np.float64))
    try:
        x = meshgen.rng_for(96, 0).standard_normal((na, 3, 2))
        y = gm.matvec_l2(to_dev(x, np.float64)).cpu().numpy()
        assert np.max(np.abs(y - 1.7 * dof_apply(A2, x))) <= 1e-12 * np.max(np.abs(y))
    finally:
        gm.set_material(to_dev(m.young, np.float64), to_dev(m.poisson, np.float64))


@pytest.fixture(scope="module")
def crust3(gpu_lib):
    m = meshgen.crust_mesh(12, 12, 6)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(3, 2), nrhs=16)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    print(f"[crust 12x12x6] DOF={m.n_dof}: oracle sparse LU", flush=True)
    return m, ebe.Mesh.from_generated(m), f, solve.sparse_solve(K, f, m.fixed)


@pytest.mark.parametrize("mode", [ebe.MODE_MIXED, ebe.MODE_FP64])
def test_crust_mg3_within_1e6(crust3, mode):
    m, gm, f, ud = crust3
    u, st = gm.solve(torch.from_numpy(f).cuda(), precond=ebe.PREC_MG3, mode=mode, tol=1e-8)
    print(f"[crust MG3 mode={mode}] {st}", flush=True)
    assert st["status"] == ebe.OK and st["max_rel_res"] <= 1e-8
    assert st["inner_iters"][2] > 0
    err = np.linalg.norm(u.cpu().numpy() - ud) / np.linalg.norm(ud)
    assert err <= 1e-6


@pytest.mark.parametrize("nrhs", [3, 7])
def test_crust_mg3_odd_case_counts(crust3, nrhs):
    """Case counts that are not powers of two (one case per work-item in the
    assembled and transfer kernels, workgroups of 3 * 85 and 7 * 36 lanes)."""
    m, gm, f, ud = crust3
    fs = np.ascontiguousarray(f[:, :, :nrhs])
    u, st = gm.solve(torch.from_numpy(fs).cuda(), precond=ebe.PREC_MG3, mode=ebe.MODE_MIXED, tol=1e-8)
    assert st["status"] == ebe.OK and st["max_rel_res"] <= 1e-8
    err = np.linalg.norm(u.cpu().numpy() - ud[:, :, :nrhs]) / np.linalg.norm(ud[:, :, :nrhs])
    assert err <= 1e-6


def test_small_mg3_matches_oracle_three_level_solve(gpu_lib):
    m = meshgen.crust_mesh(6, 6, 3)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(3, 2), nrhs=4)
    gm = ebe.Mesh.from_generated(m)
    u, st = gm.solve(torch.from_numpy(f).cuda(), precond=ebe.PREC_MG3, tol=1e-10)
    uo, sto = alg1.adaptive_cg(m.xyz, m.conn, m.n_vertices, m.young, m.poisson, m.fixed, f, tol=1e-10, levels=3)
    print(f"[crust 6x6x3 MG3] gpu {st} oracle {sto}", flush=True)
    assert st["status"] == ebe.OK
    # both converge to the same solution; iteration counts are not pinned
    assert np.linalg.norm(u.cpu().numpy() - uo) / np.linalg.norm(uo) <= 1e-8


@pytest.mark.parametrize("grid", [(1, 1, 1), (2, 1, 1), (3, 2, 2)])
def test_tiny_meshes_level2_and_mg3(gpu_lib, grid):
    """One or a few aggregates (a single slice, ragged rows): aggregates,
    A2 x and an MG3 solve against the dense solution."""
    m = meshgen.kuhn_mesh(*grid, jitter=0.1, rng=meshgen.rng_for(97, sum(grid)))
    meshgen.fix_faces(m, [(2, 0)])
    K1 = fem.assemble(m.xyz, m.conn, m.young, m.poisson, order=1, n_nodes=m.n_vertices)
    agg, na, P2, A2, cfx = amg.level2(m.conn, m.n_vertices, K1, m.fixed)
    gm = ebe.Mesh.from_generated(m)
    n, a = gm.level2_info()
    assert n == na and np.array_equal(a, agg)
    x = meshgen.rng_for(98, 0).standard_normal((na, 3, 2))
    y = gm.matvec_l2(to_dev(x, np.float64), apply_bc=True).cpu().numpy()
    xm = x.copy()
    xm[cfx] = 0
    ref = dof_apply(A2, xm)
    ref[cfx] = 0
    assert np.max(np.abs(y - ref)) <= 1e-12 * max(np.max(np.abs(ref)), 1e-300)
    f = meshgen.top_face_random_loads(m, meshgen.rng_for(98, 1), nrhs=1)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    ud = solve.dense_solve(K, f, m.fixed)
    u, st = gm.solve(torch.from_numpy(f).cuda(), precond=ebe.PREC_MG3, mode=ebe.MODE_MIXED, tol=1e-10)
    assert st["status"] == ebe.OK
    assert np.linalg.norm(u.cpu().numpy() - ud) <= 1e-8 * np.linalg.norm(ud)
