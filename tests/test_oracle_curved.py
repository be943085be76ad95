"""Pins of the oracle's stiffness on curved (isoparametric) 10-node tetrahedra:
edge nodes off their edge midpoints, the element map quadratic, its Jacobian
varying inside the element.  The oracle evaluates K_e = sum_q w_q B_q^T D B_q
|det J_q| with the 4-point rule at each point's own Jacobian (Section 2,
Eq. (2)); these facts fix it independently of its formulas.

* A straight tetrahedron T0 mapped by the global quadratic map
  phi(X) = (X1 + c X1^2, X2, X3) is represented exactly by a quadratic
  element (the interpolation of a quadratic map is the map).  A linear
  displacement u = A x then has the constant strain sym(A), so
  u^T K_e u = vol(phi(T0)) * (eps : C : eps), and
  vol(phi(T0)) = V0 (1 + 2 c mean(X1)) since det grad phi = 1 + 2 c X1 is
  linear.  The integrand det J is linear in the reference coordinates, so the
  rule is exact: the identity holds to rounding.  It fails for a per-element
  (corner) volume, a transposed Jacobian, a wrong point or weight.
* The same map applied to a whole lattice: a uniform stress is in
  equilibrium, so K applied to a linear field vanishes at every interior
  node (det J grad N is quadratic under this map, so the rule is exact).
* Any curved element: symmetric, positive semi-definite, rank 24, rigid
  motions in the null space.
The elastic constants here come from the bulk and shear moduli,
K = E / (3 (1 - 2 nu)), mu = E / (2 (1 + nu)), lambda = K - 2 mu / 3, not
from the oracle's material module.
"""
import numpy as np
import pytest

from oracle import fem
from paper_1710_08679_amd import meshgen


def straight_tet(rng, jitter=0.25):
    base = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    x = base + rng.uniform(-jitter, jitter, size=(4, 3))
    if np.linalg.det(np.stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]], axis=1)) < 0:
        x[[1, 2]] = x[[2, 1]]
    edges = np.array([(x[p] + x[q]) / 2 for p, q in meshgen.VTK_EDGES])
    return np.concatenate([x, edges])


def phi(x, c):
    y = x.copy()
    y[..., 0] = x[..., 0] + c * x[..., 0] ** 2
    return y


def energy_density(eps, E, nu):
    mu = E / (2.0 * (1.0 + nu))
    lam = E / (3.0 * (1.0 - 2.0 * nu)) - 2.0 * mu / 3.0
    return lam * np.trace(eps) ** 2 + 2.0 * mu * np.sum(eps * eps)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("c", [0.0, 0.25, -0.3])
def test_mapped_element_energy_of_linear_fields(seed, c):
    rng = np.random.default_rng(seed + 40)
    X = straight_tet(rng)
    x = phi(X, c)
    E, nu = 1.0 + 2.0 * rng.random(), 0.1 + 0.35 * rng.random()
    K = fem.element_stiffness_p2(x[None], E, nu)[0]
    v0 = np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)) / 6.0
    vol = v0 * (1.0 + 2.0 * c * X[:4, 0].mean())
    for _ in range(3):
        A = rng.standard_normal((3, 3))
        u = (x @ A.T).ravel()  # node-major (x, y, z)
        want = vol * energy_density(0.5 * (A + A.T), E, nu)
        assert u @ K @ u == pytest.approx(want, rel=1e-12)
        if c != 0.0:
            # the curvature matters: the straight element through the same corners differs
            xs = np.concatenate([x[:4], [(x[p] + x[q]) / 2 for p, q in meshgen.VTK_EDGES]])
            Ks = fem.element_stiffness_p2(xs[None], E, nu)[0]
            us = (xs @ A.T).ravel()
            assert abs(us @ Ks @ us - want) > 1e-4 * abs(want)


def test_mapped_lattice_linear_field_is_equilibrated_at_interior_nodes():
    m = meshgen.quadratic_map(meshgen.kuhn_mesh(4, 4, 4, jitter=0.2, rng=meshgen.rng_for(90, 5)), 0.3)
    mid = 0.5 * (m.xyz[m.conn[:, [p for p, _ in meshgen.VTK_EDGES]]] + m.xyz[m.conn[:, [q for _, q in meshgen.VTK_EDGES]]])
    assert np.abs(m.xyz[m.conn[:, 4:]] - mid).max() > 1e-3  # the elements are curved
    A = np.random.default_rng(7).standard_normal((3, 3))
    u = (m.xyz @ A.T)[:, :, None]
    y = fem.ebe_apply(m.xyz, m.conn, 2.0, 0.3, u)[:, :, 0]
    r = m.refined
    inner = np.all((r > 0) & (r < 2 * np.array(m.grid)), axis=1)
    assert np.abs(y[inner]).max() <= 1e-12 * np.abs(y).max()
    assert np.abs(y[~inner]).max() > 1e-3 * np.abs(y).max()


@pytest.mark.parametrize("seed", range(4))
def test_curved_element_symmetric_psd_rank24_rigid_null(seed):
    m = meshgen.curve_edges(meshgen.kuhn_mesh(2, 2, 2, jitter=0.2, rng=meshgen.rng_for(90, seed)),
                            meshgen.rng_for(91, seed), amp=0.12)
    xe = m.xyz[m.conn]
    K = fem.element_stiffness_p2(xe, 1.5, 0.3)
    for e in range(0, m.n_elem, 7):
        k = K[e]
        scale = np.abs(k).max()
        assert np.abs(k - k.T).max() <= 1e-14 * scale
        w = np.linalg.eigvalsh(k)
        assert w.min() >= -1e-12 * scale
        assert np.sum(w > 1e-9 * scale) == 24
        x = xe[e]
        modes = [np.tile(np.eye(3)[d], 10) for d in range(3)]
        modes += [np.cross(np.eye(3)[d], x).ravel() for d in range(3)]
        for r in modes:
            assert np.abs(k @ r).max() <= 1e-12 * scale * np.abs(r).max()
