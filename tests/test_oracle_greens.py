"""Pins of the oracle's Green's-function pipeline (Section 5, Eq. (4)-(5);
split-node fault loading, Section 2).

* Split node: a fault plane that cuts the whole mesh in two, with one block
  clamped and the other free, turns any rigid relative motion into a known
  displacement field: the free block moves rigidly by the slip, the clamped
  one stays, and the fault nodes carry the mean (half the slip).  Uniform
  slip and a rigid rotation both reproduce it to rounding, which fixes the
  sign of each side and the factor 1/2.
* The cubic B-spline basis: partition of unity and support.
* Inversion: noise-free data from a known slip is recovered; the solution
  meets the first-order optimality condition of Eq. (5); the curvature
  routine gives 1/R on a circle; on a synthetic ill-posed problem the L-curve
  corner lands near the best regularisation of the grid.
"""
import numpy as np
import pytest

from oracle import fem, greens, solve
from paper_1710_08679_amd import meshgen


def cut_mesh():
    """Unit cube, 4^3 hexes; the plane y - z = h cuts it in two; the face y = 0
    (all on the y - z < h side) is clamped; the other block is free."""
    m = meshgen.kuhn_mesh(4, 4, 4, jitter=0.0)
    meshgen.set_layers_flat(m)
    m.fixed[meshgen.face_nodes(m, 1, 0), :] = 1
    r = m.refined
    k = 2  # refined units: y - z = h
    plane = (r[:, 1] - r[:, 2]) == k
    plus = (r[:, 1] - r[:, 2]) > k
    d = (r[m.conn[:, :4], 1] - r[m.conn[:, :4], 2] - k).sum(axis=1)
    sides = np.where(plane[m.conn].any(axis=1), np.sign(d), 0).astype(np.int8)
    return m, plane, plus, sides


@pytest.mark.parametrize("kind", ["uniform", "rotation"])
def test_split_node_rigid_block(kind):
    m, plane, plus, sides = cut_mesh()
    assert not m.fixed[plane | plus].any()
    if kind == "uniform":
        motion = np.tile(np.array([0.3, -0.2, 0.5]), (m.n_nodes, 1))
    else:
        w, x0 = np.array([0.2, -0.1, 0.15]), np.array([0.5, 0.5, 0.5])
        motion = np.cross(w, m.xyz - x0)
    slip = np.zeros((m.n_nodes, 3, 1))
    slip[plane, :, 0] = motion[plane]                   # u+ - u- = rigid motion on the fault
    f = greens.split_node_forces(m.xyz, m.conn, m.young, m.poisson, sides, slip)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    v = solve.sparse_solve(K, f, m.fixed)[:, :, 0]
    exact = np.zeros((m.n_nodes, 3))
    exact[plus] = motion[plus]
    exact[plane] = 0.5 * motion[plane]
    assert np.abs(v - exact).max() <= 1e-10 * np.abs(motion).max()
    # a wrong side sign, or a missing 1/2, is far from it
    bad = greens.split_node_forces(m.xyz, m.conn, m.young, m.poisson, -sides, slip)
    vb = solve.sparse_solve(K, bad, m.fixed)[:, :, 0]
    assert np.abs(vb - exact).max() > 0.1 * np.abs(motion).max()


def test_cubic_bspline_partition_of_unity_and_support():
    t = np.linspace(-3.0, 3.0, 601)
    total = sum(meshgen.cubic_bspline(t - i) for i in range(-6, 7))
    assert np.abs(total - 1.0).max() <= 1e-14
    assert np.all(meshgen.cubic_bspline(np.array([-2.0, 2.0, 2.5, -7.0])) == 0.0)
    assert meshgen.cubic_bspline(np.array([0.0]))[0] == pytest.approx(2.0 / 3.0)


def test_fault_patch_geometry():
    """Fault nodes are the plane's nodes inside the patch; each basis function
    is a tensor-product cubic B-spline in (x, eta) whose support lies inside
    the patch; elements touching the fault lie on one side of the plane."""
    m = meshgen.crust_mesh(12, 12, 6)
    flt = meshgen.dipping_fault(m, 0.5, (0.3, 1.7), (0.566, 1.556), (4, 2))
    x, eta = m.xyz[:, 0], (m.xyz[:, 1] + m.xyz[:, 2]) / np.sqrt(2.0)
    on = np.isclose(m.xyz[:, 1] - m.xyz[:, 2], 0.5)
    want = np.nonzero(on & (x >= 0.3) & (x <= 1.7) & (eta >= 0.566) & (eta <= 1.556))[0]
    assert np.array_equal(np.sort(flt.nodes), want)
    ns, nd = flt.knots
    hs, hd = 1.4 / (ns + 3), (1.556 - 0.566) / (nd + 3)
    for i in range(ns):
        for j in range(nd):
            b = meshgen.cubic_bspline((flt.coords[:, 0] - 0.3 - hs * (2 + i)) / hs) * \
                meshgen.cubic_bspline((flt.coords[:, 1] - 0.566 - hd * (2 + j)) / hd)
            assert np.allclose(flt.basis[:, i * nd + j], b, rtol=0, atol=1e-15)
            assert np.allclose(flt.basis[:, ns * nd + i * nd + j], b, rtol=0, atol=1e-15)
    assert np.allclose(flt.dirs[:ns * nd], [1, 0, 0]) and np.allclose(flt.dirs[ns * nd:], np.array([0, 1, 1]) / 2 ** 0.5)
    r = m.refined
    assert np.all(r[flt.nodes, 1] - r[flt.nodes, 2] == flt.k)
    # every element with a fault node lies on one side of the plane
    dv = r[m.conn[:, :4], 1] - r[m.conn[:, :4], 2] - flt.k
    touch = flt.sides != 0
    assert np.all((dv[touch] >= 0).all(axis=1) | (dv[touch] <= 0).all(axis=1))


@pytest.fixture(scope="module")
def small_greens():
    m = meshgen.crust_mesh(12, 12, 6)
    flt = meshgen.dipping_fault(m, 0.5, (0.3, 1.7), (0.566, 1.556), (4, 2))
    st = meshgen.surface_stations(m, 1)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    slip = flt.slip(m.n_nodes, np.arange(flt.n_basis))
    f = greens.split_node_forces(m.xyz, m.conn, m.young, m.poisson, flt.sides, slip)
    u = solve.sparse_solve(K, f, m.fixed)
    return m, flt, st, greens.greens_matrix(u, st)


def test_noise_free_slip_is_recovered(small_greens):
    m, flt, st, G = small_greens
    a_true = meshgen.rng_for(6, 0).standard_normal(flt.n_basis)
    d = G @ a_true
    L = greens.smoothing_matrix(*flt.knots)
    a = greens.regularized_lsq(G, d, L, 1e-9 * np.linalg.norm(G, 2))
    assert np.abs(a - a_true).max() <= 1e-6 * np.abs(a_true).max()


def test_regularized_solution_is_stationary(small_greens):
    m, flt, st, G = small_greens
    d = G @ meshgen.rng_for(6, 1).standard_normal(flt.n_basis) + 1e-3 * meshgen.rng_for(6, 2).standard_normal(
        G.shape[0])
    L = greens.smoothing_matrix(*flt.knots)
    alpha = 0.05 * np.linalg.norm(G, 2)
    a = greens.regularized_lsq(G, d, L, alpha)
    grad = G.T @ (G @ a - d) + alpha ** 2 * (L.T @ (L @ a))
    assert np.abs(grad).max() <= 1e-10 * np.abs(G.T @ d).max()


def test_curvature_of_a_circle():
    t = np.linspace(0.2, 2.5, 400)
    R = 3.0
    k = greens.curvature(R * np.cos(t), R * np.sin(t), t)
    assert np.abs(k[2:-2] - 1.0 / R).max() <= 1e-4


def test_l_curve_corner_is_near_the_best_alpha():
    """Synthetic ill-posed problem: singular values decaying over eight
    decades, data noise at 1e-4.  The corner's solution error is within a
    factor 3 of the smallest error over the alpha grid."""
    rng = meshgen.rng_for(6, 3)
    n = 40
    U, _ = np.linalg.qr(rng.standard_normal((60, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0, -8, n)
    G = (U * s) @ V.T
    a_true = V @ (s ** 0.5 * rng.standard_normal(n))  # satisfies the discrete Picard condition
    d = G @ a_true + 1e-4 * rng.standard_normal(60) / np.sqrt(60)
    L = np.eye(n)
    alphas = np.logspace(-9, 0, 91)
    rho, eta, sols, k, _ = greens.l_curve(G, d, L, alphas)
    assert np.all(np.diff(rho) >= -1e-12 * rho[:-1]) and np.all(np.diff(eta) <= 1e-12 * eta[:-1])
    err = np.linalg.norm(sols - a_true[None, :], axis=1)
    assert err[k] <= 3.0 * err.min()
