"""Pins of the oracle's element stiffness against facts fixed by elasticity
theory, independent of the oracle's own formulas.

* Bilinear-form identity: for any two quadratic displacement fields (which a
  10-node tetrahedron represents exactly) u_e^T K_e v_e must equal the strain
  energy integral of eps(u) : C : eps(v) (Section 2, Eq. (1a-b)).  The reference
  integral here uses analytic strains of polynomial fields, the tensor (not
  Voigt) form of C, and a collapsed Gauss-Legendre rule from numpy; since the
  30 nodal values span all quadratic fields, this fixes every entry of K_e.
* Rigid-body modes, symmetry, PSD, rank 24.
* Rotation covariance (isotropy) and length scaling.
"""
import numpy as np
import pytest

from oracle import fem, material
from paper_1710_08679_amd import meshgen


def random_tet(rng, jitter=0.25):
    base = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    x = base + rng.uniform(-jitter, jitter, size=(4, 3))
    if np.linalg.det(np.stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]], axis=1)) < 0:
        x[[1, 2]] = x[[2, 1]]
    edges = np.array([(x[p] + x[q]) / 2 for p, q in meshgen.VTK_EDGES])
    return np.concatenate([x, edges])


MONO = [lambda x: np.ones(len(x)), lambda x: x[:, 0], lambda x: x[:, 1], lambda x: x[:, 2],
        lambda x: x[:, 0] ** 2, lambda x: x[:, 1] ** 2, lambda x: x[:, 2] ** 2,
        lambda x: x[:, 0] * x[:, 1], lambda x: x[:, 1] * x[:, 2], lambda x: x[:, 2] * x[:, 0]]


def mono_grad(x):
    """(len(x), 10, 3) analytic gradients of the monomials above."""
    g = np.zeros((len(x), 10, 3))
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    g[:, 1, 0] = 1
    g[:, 2, 1] = 1
    g[:, 3, 2] = 1
    g[:, 4, 0] = 2 * X
    g[:, 5, 1] = 2 * Y
    g[:, 6, 2] = 2 * Z
    g[:, 7, 0], g[:, 7, 1] = Y, X
    g[:, 8, 1], g[:, 8, 2] = Z, Y
    g[:, 9, 2], g[:, 9, 0] = X, Z
    return g


def collapsed_rule(x4, npts=6):
    """Points/weights on a physical tetrahedron by the collapsed (Duffy)
    map of a Gauss-Legendre tensor rule on the unit cube."""
    t, w = np.polynomial.legendre.leggauss(npts)
    t = 0.5 * (t + 1)
    w = 0.5 * w
    S, T, W = np.meshgrid(t, t, t, indexing="ij")
    WS, WT, WW = np.meshgrid(w, w, w, indexing="ij")
    a = S.ravel()
    b = (1 - S.ravel()) * T.ravel()
    c = (1 - S.ravel()) * (1 - T.ravel()) * W.ravel()
    jac = (1 - S.ravel()) ** 2 * (1 - T.ravel())
    J = np.stack([x4[1] - x4[0], x4[2] - x4[0], x4[3] - x4[0]], axis=1)
    pts = x4[0] + np.stack([a, b, c], axis=1) @ J.T
    wts = (WS * WT * WW).ravel() * jac * abs(np.linalg.det(J))
    return pts, wts


def energy_form(coef_u, coef_v, x4, E, nu):
    """int eps(u):C:eps(v) dV for fields u_c(x) = sum_k coef[k, c] m_k(x)."""
    pts, wts = collapsed_rule(x4)
    g = mono_grad(pts)
    Gu = np.einsum("pkd,kc->pcd", g, coef_u)  # du_c/dx_d
    Gv = np.einsum("pkd,kc->pcd", g, coef_v)
    eu = 0.5 * (Gu + Gu.transpose(0, 2, 1))
    ev = 0.5 * (Gv + Gv.transpose(0, 2, 1))
    lam, mu = material.lame(E, nu)
    tr_u = np.trace(eu, axis1=1, axis2=2)
    tr_v = np.trace(ev, axis1=1, axis2=2)
    dens = lam * tr_u * tr_v + 2 * mu * np.einsum("pij,pij->p", eu, ev)
    return float(np.sum(wts * dens))


def nodal(coef, xe):
    vals = np.stack([m(xe) for m in MONO], axis=1)  # (10 nodes, 10 monomials)
    return (vals @ coef).ravel()  # node-major (x, y, z)


@pytest.mark.parametrize("seed", range(5))
def test_p2_stiffness_equals_strain_energy_of_quadratic_fields(seed):
    rng = np.random.default_rng(100 + seed)
    xe = random_tet(rng)
    E, nu = rng.uniform(0.5, 5.0), rng.uniform(0.0, 0.45)
    Ke = fem.element_stiffness_p2(xe[None], np.array([E]), np.array([nu]))[0]
    for _ in range(4):
        cu = rng.standard_normal((10, 3))
        cv = rng.standard_normal((10, 3))
        ref = energy_form(cu, cv, xe[:4], E, nu)
        got = nodal(cu, xe) @ Ke @ nodal(cv, xe)
        assert abs(got - ref) <= 1e-12 * (abs(ref) + np.abs(Ke).max())


@pytest.mark.parametrize("seed", range(3))
def test_p1_stiffness_equals_strain_energy_of_linear_fields(seed):
    rng = np.random.default_rng(200 + seed)
    xe = random_tet(rng)[:4]
    E, nu = rng.uniform(0.5, 5.0), rng.uniform(0.0, 0.45)
    Ke = fem.element_stiffness_p1(xe[None], np.array([E]), np.array([nu]))[0]
    for _ in range(4):
        cu = np.zeros((10, 3))
        cv = np.zeros((10, 3))
        cu[:4] = rng.standard_normal((4, 3))
        cv[:4] = rng.standard_normal((4, 3))
        ref = energy_form(cu, cv, xe, E, nu)
        vu = (np.stack([m(xe) for m in MONO[:4]], axis=1) @ cu[:4]).ravel()
        vv = (np.stack([m(xe) for m in MONO[:4]], axis=1) @ cv[:4]).ravel()
        assert abs(vu @ Ke @ vv - ref) <= 1e-12 * (abs(ref) + np.abs(Ke).max())


def rigid_modes(xe):
    n = len(xe)
    modes = []
    for c in range(3):
        t = np.zeros((n, 3))
        t[:, c] = 1
        modes.append(t.ravel())
    for w in np.eye(3):
        modes.append(np.cross(w, xe).ravel())
    return np.stack(modes, axis=1)


@pytest.mark.parametrize("seed", range(5))
def test_p2_stiffness_symmetric_psd_rank24_rigid_null(seed):
    rng = np.random.default_rng(300 + seed)
    xe = random_tet(rng)
    Ke = fem.element_stiffness_p2(xe[None], np.array([2.0]), np.array([0.3]))[0]
    scale = np.abs(Ke).max()
    assert np.abs(Ke - Ke.T).max() <= 1e-14 * scale
    ev = np.linalg.eigvalsh(Ke)
    assert ev.min() >= -1e-12 * scale
    assert np.sum(ev > 1e-10 * scale) == 24
    assert np.abs(Ke @ rigid_modes(xe)).max() <= 1e-13 * scale


def test_p2_stiffness_rotation_covariant_and_scales_with_length():
    rng = np.random.default_rng(7)
    xe = random_tet(rng)
    Ke = fem.element_stiffness_p2(xe[None], np.array([1.3]), np.array([0.27]))[0]
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    KR = fem.element_stiffness_p2((xe @ Q.T)[None], np.array([1.3]), np.array([0.27]))[0]
    B = np.kron(np.eye(10), Q)
    assert np.allclose(KR, B @ Ke @ B.T, atol=1e-13 * np.abs(Ke).max())
    Ks = fem.element_stiffness_p2((2.5 * xe)[None], np.array([1.3]), np.array([0.27]))[0]
    assert np.allclose(Ks, 2.5 * Ke, rtol=0, atol=1e-13 * np.abs(Ks).max())


def test_stiffness_linear_in_young_modulus():
    rng = np.random.default_rng(8)
    xe = random_tet(rng)
    K1 = fem.element_stiffness_p2(xe[None], np.array([1.0]), np.array([0.3]))[0]
    K7 = fem.element_stiffness_p2(xe[None], np.array([7.0]), np.array([0.3]))[0]
    assert np.allclose(K7, 7.0 * K1, rtol=1e-14, atol=1e-14 * np.abs(K7).max())


def test_table3_wave_speeds_round_trip():
    """Table 3 gives layers as (Vp, Vs, rho); mu = rho Vs^2 and lambda + 2 mu = rho Vp^2."""
    for vp, vs, rho in meshgen.PAPER_TABLE3:
        E, nu = material.from_wave_speeds(vp, vs, rho)
        lam, mu = material.lame(E, nu)
        assert np.isclose(mu, rho * vs ** 2, rtol=1e-13)
        assert np.isclose(lam + 2 * mu, rho * vp ** 2, rtol=1e-13)
        assert 0 < nu < 0.5


def test_table3_golden_fixture_matches_generator():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table3_materials.json")))
    assert tuple((l["vp"], l["vs"], l["rho"]) for l in g["layers"]) == meshgen.PAPER_TABLE3
