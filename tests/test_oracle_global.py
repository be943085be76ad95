"""Pins of the oracle's global operator and solves.

* Global K: symmetric; annihilates rigid motions of the whole mesh.
* EBE product by definition (Eq. (3)) equals the assembled CSR product, and
  an element-by-element brute force on a tiny mesh.
* Homogeneous material, jittered mesh: K applied to a linear field vanishes at
  every interior node (a uniform stress is in equilibrium).
* Patch test: prescribing a linear field on the boundary reproduces it inside.
* Uniaxial bar: rollers on three faces and a consistent uniform traction give
  u = (s x / E, -nu s y / E, -nu s z / E) exactly.
* Dense Cholesky, sparse LU and block-Jacobi CG agree; multi-RHS equals
  column-by-column.
* P1 (quadratic <- linear) reproduces linear fields at all nodes.
"""
import numpy as np
import pytest

from oracle import fem, solve, alg1
from paper_1710_08679_amd import meshgen


def small_mesh(g=3, jitter=0.2, seed=0, lengths=(1.0, 1.0, 1.0), grid=None):
    a, b, c = grid if grid is not None else (g, g, g)
    return meshgen.kuhn_mesh(a, b, c, lengths=lengths, jitter=jitter, rng=meshgen.rng_for(90, seed))


def test_mesh_generator_counts_and_orientation():
    m = meshgen.kuhn_mesh(4, 3, 2)
    assert m.n_elem == 6 * 4 * 3 * 2
    assert m.n_nodes == 9 * 7 * 5
    assert m.n_vertices == 5 * 4 * 3
    x, c = m.xyz, m.conn
    d = np.linalg.det(np.stack([x[c[:, 1]] - x[c[:, 0]], x[c[:, 2]] - x[c[:, 0]], x[c[:, 3]] - x[c[:, 0]]], axis=2))
    assert d.min() > 0
    assert np.isclose(d.sum() / 6, 1.0)
    assert c[:, :4].max() < m.n_vertices and c[:, 4:].min() >= m.n_vertices


def test_global_symmetric_and_rigid_null():
    m = small_mesh()
    meshgen.set_layers_flat(m)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    s = abs(K).max()
    assert abs(K - K.T).max() <= 1e-14 * s
    for c in range(3):
        t = np.zeros((m.n_nodes, 3))
        t[:, c] = 1
        assert np.abs(K @ t.ravel()).max() <= 1e-13 * s
    for w in np.eye(3):
        rot = np.cross(w, m.xyz).ravel()
        assert np.abs(K @ rot).max() <= 1e-13 * s


def test_ebe_definition_matches_assembled_and_brute_force():
    m = small_mesh(g=2)
    meshgen.set_layers_flat(m)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((m.n_nodes, 3, 3))
    y = fem.ebe_apply(m.xyz, m.conn, m.young, m.poisson, x)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    y2 = (K @ x.reshape(-1, 3)).reshape(m.n_nodes, 3, 3)
    assert np.abs(y - y2).max() <= 1e-13 * np.abs(y).max()
    # brute force: a python loop over elements and local rows
    y3 = np.zeros_like(x)
    for e in range(m.n_elem):
        Ke = fem.element_stiffness_p2(m.xyz[m.conn[e]][None], m.young[e:e + 1], m.poisson[e:e + 1])[0]
        for a in range(10):
            for ca in range(3):
                for b in range(10):
                    for cb in range(3):
                        y3[m.conn[e, a], ca] += Ke[3 * a + ca, 3 * b + cb] * x[m.conn[e, b], cb]
    assert np.abs(y - y3).max() <= 1e-13 * np.abs(y).max()


def test_linear_field_is_equilibrated_at_interior_nodes():
    m = small_mesh(g=4, jitter=0.2, seed=2)
    rng = np.random.default_rng(2)
    eps = rng.standard_normal((3, 3))
    u = (m.xyz @ eps.T)[:, :, None]
    y = fem.ebe_apply(m.xyz, m.conn, 2.0, 0.3, u)[:, :, 0]
    r = m.refined
    inner = np.all((r > 0) & (r < 2 * np.array(m.grid)), axis=1)
    assert np.abs(y[inner]).max() <= 1e-12 * np.abs(y).max()
    assert np.abs(y[~inner]).max() > 1e-3 * np.abs(y).max()  # boundary tractions are not zero


def boundary_nodes(m):
    r = m.refined
    return ~np.all((r > 0) & (r < 2 * np.array(m.grid)), axis=1)


def test_patch_test_reproduces_linear_field():
    m = small_mesh(g=4, jitter=0.2, seed=3)
    rng = np.random.default_rng(3)
    eps = 1e-3 * rng.standard_normal((3, 3))
    c0 = rng.standard_normal(3)
    exact = (m.xyz @ eps.T + c0)[:, :, None]
    fixed = np.zeros((m.n_nodes, 3), np.uint8)
    fixed[boundary_nodes(m)] = 1
    K = fem.assemble(m.xyz, m.conn, 1.7, 0.28)
    u = solve.sparse_solve(K, np.zeros_like(exact), fixed, u_fixed=exact)
    assert np.abs(u - exact).max() <= 1e-12 * np.abs(exact).max()


def consistent_face_traction(m, axis, side, traction):
    """Nodal forces of a uniform traction vector on a domain face: on each
    6-node boundary triangle, corners get 0 and mid-edge nodes get A/3 each."""
    lim = 0 if side == 0 else 2 * m.grid[axis]
    on = m.refined[:, axis] == lim
    f = np.zeros((m.n_nodes, 3, 1))
    faces = ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))
    edge_of = {tuple(sorted(e)): 4 + k for k, e in enumerate(meshgen.VTK_EDGES)}
    seen = set()
    for e in range(m.n_elem):
        c = m.conn[e]
        for tri in faces:
            vs = c[list(tri)]
            if not on[vs].all():
                continue
            key = tuple(sorted(vs))
            if key in seen:
                continue
            seen.add(key)
            x = m.xyz[vs]
            A = 0.5 * np.linalg.norm(np.cross(x[1] - x[0], x[2] - x[0]))
            for p, q in ((0, 1), (1, 2), (0, 2)):
                node = c[edge_of[tuple(sorted((tri[p], tri[q])))]]
                f[node, :, 0] += np.asarray(traction) * A / 3.0
    return f


@pytest.mark.parametrize("jitter", [0.0, 0.2])
def test_uniaxial_bar_closed_form(jitter):
    m = small_mesh(grid=(4, 2, 2), lengths=(2.0, 1.0, 1.0), jitter=jitter, seed=4)
    E, nu, s0 = 2.5, 0.3, 0.7
    for axis in range(3):
        m.fixed[meshgen.face_nodes(m, axis, 0), axis] = 1
    f = consistent_face_traction(m, 0, 1, (s0, 0.0, 0.0))
    assert np.isclose(f.sum(), s0 * 1.0 * 1.0)
    K = fem.assemble(m.xyz, m.conn, E, nu)
    u = solve.sparse_solve(K, f, m.fixed)
    X = m.xyz
    exact = np.stack([s0 * X[:, 0] / E, -nu * s0 * X[:, 1] / E, -nu * s0 * X[:, 2] / E], axis=1)
    assert np.abs(u[:, :, 0] - exact).max() <= 1e-12 * np.abs(exact).max()


def test_dense_sparse_cg_agree_and_multi_rhs_is_columnwise():
    m = meshgen.cube_mesh(4)
    f = meshgen.top_face_random_loads(m, meshgen.rng_for(1, 0), nrhs=3)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    ud = solve.dense_solve(K, f, m.fixed)
    us = solve.sparse_solve(K, f, m.fixed)
    uc, its = solve.pcg(K, f, m.fixed, tol=1e-13)
    sc = np.abs(ud).max()
    assert np.abs(ud - us).max() <= 1e-12 * sc
    assert np.abs(ud - uc).max() <= 1e-9 * sc
    assert np.all(ud[m.fixed.astype(bool)] == 0)
    for j in range(3):
        uj = solve.dense_solve(K, f[:, :, j:j + 1], m.fixed)
        assert np.abs(uj[:, :, 0] - ud[:, :, j]).max() <= 1e-12 * sc
    r = solve.residual(K, ud, f, m.fixed)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(f)


def test_p1_prolongation_reproduces_linear_fields():
    m = small_mesh(g=3, jitter=0.2, seed=5)
    P = fem.prolongation_p1(m.conn, m.n_nodes, m.n_vertices)
    rng = np.random.default_rng(5)
    A = rng.standard_normal((3, 3))
    lin = m.xyz @ A.T
    got = fem.apply_scalar_op(P, lin[:m.n_vertices, :, None])[:, :, 0]
    assert np.abs(got - lin).max() <= 1e-13 * np.abs(lin).max()
    assert np.allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0)
    assert P.nnz == m.n_vertices + 2 * (m.n_nodes - m.n_vertices)


@pytest.mark.parametrize("coarse_guess", ["restrict", "inject"])
def test_algorithm1_converges_to_direct_solution(coarse_guess):
    m = meshgen.crust_mesh(6, 6, 3)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(3, 2), nrhs=4)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    ud = solve.sparse_solve(K, f, m.fixed)
    u, st = alg1.adaptive_cg(m.xyz, m.conn, m.n_vertices, m.young, m.poisson, m.fixed, f, tol=1e-10,
                             coarse_guess=coarse_guess)
    assert st["max_rel_res"] <= 1e-10
    err = np.linalg.norm(u - ud) / np.linalg.norm(ud)
    assert err <= 1e-7
