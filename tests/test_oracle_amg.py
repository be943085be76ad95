"""Pins of the oracle's level 2 (algebraic coarsening of the linear mesh).

* Aggregation, by hand on paths, a star and a small tree, and structurally on
  a mesh: a partition of the corners into connected aggregates, each holding
  a corner together with its whole neighbourhood.
* Smoothed prolongator: maps a coarse translation to the fine translation
  without Dirichlet conditions (K1 annihilates it, so the smoothing step
  leaves it); empty rows at fixed DOFs; omega = 0 gives the 0/1 tentative map.
* Galerkin A2: symmetric; without Dirichlet conditions it annihilates the
  three coarse translations; with one-corner aggregates and omega = 0 it is
  P K1 P (the fixed DOFs' rows and columns removed); positive definite on
  the free coarse DOFs of a clamped mesh.
* Three-level Algorithm 1 converges to the direct solution.
"""
import numpy as np
import scipy.sparse as sp

from oracle import alg1, amg, fem, solve
from paper_1710_08679_amd import meshgen


def path(n):
    return [np.array([u for u in (v - 1, v + 1) if 0 <= u < n]) for v in range(n)]


def test_aggregation_by_hand():
    # path 0-1-2-3-4-5-6: 0 roots {0,1}; 2 has an aggregated neighbour; 3
    # roots {2,3,4}; 5 has one; 6 roots {5,6}
    agg, na = amg.aggregate(path(7))
    assert na == 3 and agg.tolist() == [0, 0, 1, 1, 1, 2, 2]
    # path of 4: 0 roots {0,1}; 2 has an aggregated neighbour; 3's only
    # neighbour 2 is still free, so 3 roots {2,3}
    agg, na = amg.aggregate(path(4))
    assert na == 2 and agg.tolist() == [0, 0, 1, 1]
    # pass 2: path 0-1-2 with pendants 3 (on 1) and 4 (on 2): 0 roots {0,1};
    # 2 and 3 have an aggregated neighbour; 4 roots {2,4}; 3 then joins the
    # lowest aggregate among its neighbours' pass-1 aggregates (0)
    g = [np.array([1]), np.array([0, 2, 3]), np.array([1, 4]), np.array([1]), np.array([2])]
    agg, na = amg.aggregate(g)
    assert na == 2 and agg.tolist() == [0, 0, 1, 0, 1]
    # star with centre 2: 0 roots {0,2}; 1, 3, 4 join it
    star = [np.array([2]), np.array([2]), np.array([0, 1, 3, 4]), np.array([2]), np.array([2])]
    agg, na = amg.aggregate(star)
    assert na == 1 and agg.tolist() == [0, 0, 0, 0, 0]


def mesh(g=4, jitter=0.2, seed=0):
    return meshgen.kuhn_mesh(g, g, g, jitter=jitter, rng=meshgen.rng_for(91, seed))


def test_aggregation_partitions_into_connected_aggregates():
    m = mesh(5)
    nb = amg.corner_graph(m.conn, m.n_vertices)
    agg, na = amg.aggregate(nb)
    assert agg.min() == 0 and agg.max() == na - 1 and len(np.unique(agg)) == na
    for a in range(na):
        mem = np.nonzero(agg == a)[0]
        seen = {mem[0]}
        todo = [mem[0]]
        while todo:
            v = todo.pop()
            for u in nb[v]:
                if agg[u] == a and u not in seen:
                    seen.add(u)
                    todo.append(u)
        assert len(seen) == mem.size
    # every aggregate holds a corner whose whole neighbourhood lies in it
    # (its pass-1 root), so every aggregate has at least two corners
    closed = np.array([np.all(agg[nb[v]] == agg[v]) for v in range(m.n_vertices)])
    assert np.all(np.bincount(agg[closed], minlength=na) >= 1)
    assert np.bincount(agg).min() >= 2
    assert 4 <= m.n_vertices / na <= 40


def test_galerkin_null_space_and_symmetry():
    m = mesh(4)
    K1 = fem.assemble(m.xyz, m.conn, m.young, m.poisson, order=1, n_nodes=m.n_vertices)
    free = np.zeros((m.n_nodes, 3), dtype=bool)
    agg, na, P2, A2, cfx = amg.level2(m.conn, m.n_vertices, K1, free)
    assert not cfx.any()
    d = (A2 - A2.T).tocsr()
    assert abs(d).max() <= 1e-13 * abs(A2).max()
    for c in range(3):
        t = np.zeros(3 * na)
        t[c::3] = 1.0
        assert np.abs(A2 @ t).max() <= 1e-11 * abs(A2).max()
    # the same for P2 itself: a coarse constant is a fine constant
    t = np.zeros(3 * na)
    t[0::3] = 1.0
    assert np.max(np.abs(P2 @ t - np.tile([1.0, 0.0, 0.0], m.n_vertices))) <= 1e-13
    T = amg.prolongation_p2(agg, na, free)
    assert np.array_equal(T @ t, np.tile([1.0, 0.0, 0.0], m.n_vertices))
    assert (P2 - T).nnz > 0  # the smoothing step reaches neighbouring aggregates


def test_smoothed_prolongator_rows_and_omega_zero():
    m = mesh(4)
    meshgen.fix_faces(m, [(2, 0)])
    K1 = fem.assemble(m.xyz, m.conn, m.young, m.poisson, order=1, n_nodes=m.n_vertices)
    agg, na, P2, A2, cfx = amg.level2(m.conn, m.n_vertices, K1, m.fixed)
    fx = m.fixed[:m.n_vertices].astype(bool).ravel()
    assert abs(P2[np.nonzero(fx)[0]]).max() == 0
    _, _, T, A0, _ = amg.level2(m.conn, m.n_vertices, K1, m.fixed, omega=0.0)
    assert np.array_equal(T.toarray(), amg.prolongation_p2(agg, na, m.fixed).toarray())
    # each fine row of P2 touches only the aggregates of the corner's neighbours
    nb = amg.corner_graph(m.conn, m.n_vertices)
    P = P2.tocsr()
    for v in range(0, m.n_vertices, 7):
        cols = set((P.indices[P.indptr[3 * v]:P.indptr[3 * v + 3]] // 3).tolist())
        assert cols <= set(agg[np.append(nb[v], v)].tolist())


def test_galerkin_with_singleton_aggregates_is_projected_k1():
    m = mesh(3)
    meshgen.fix_faces(m, [(2, 0)])
    K1 = fem.assemble(m.xyz, m.conn, m.young, m.poisson, order=1, n_nodes=m.n_vertices)
    agg = np.arange(m.n_vertices)
    P2 = amg.prolongation_p2(agg, m.n_vertices, m.fixed)
    A2 = amg.galerkin(amg.projected(K1, m.fixed), P2)
    keep = ~m.fixed[:m.n_vertices].astype(bool).ravel()
    D = sp.diags(keep.astype(float))
    ref = (D @ K1 @ D).tocsr()
    assert abs(A2 - ref).max() <= 1e-14 * abs(ref).max()


def test_galerkin_positive_definite_on_free_coarse_dofs():
    m = mesh(4)
    meshgen.fix_faces(m, [(2, 0)])
    m.fixed[meshgen.face_nodes(m, 0, 1), 1] = 1  # one component only on another face
    K1 = fem.assemble(m.xyz, m.conn, m.young, m.poisson, order=1, n_nodes=m.n_vertices)
    agg, na, P2, A2, cfx = amg.level2(m.conn, m.n_vertices, K1, m.fixed)
    keep = ~cfx.ravel()
    A = A2.toarray()[np.ix_(keep, keep)]
    assert np.linalg.eigvalsh(A).min() > 1e-10 * np.abs(A).max()
    gone = cfx.ravel()
    assert np.all(A2.toarray()[gone] == 0) and np.all(A2.toarray()[:, gone] == 0)


def test_three_level_algorithm1_converges_to_direct_solution():
    m = meshgen.crust_mesh(6, 6, 3)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(3, 2), nrhs=4)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    ud = solve.sparse_solve(K, f, m.fixed)
    u, st = alg1.adaptive_cg(m.xyz, m.conn, m.n_vertices, m.young, m.poisson, m.fixed, f, tol=1e-10, levels=3)
    assert st["max_rel_res"] <= 1e-10 and len(st["inner"]) == 3 and st["inner"][2] > 0
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) <= 1e-7
