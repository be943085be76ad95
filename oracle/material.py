"""Isotropic linear-elastic material (Section 2, Eq. (1b); Table 3).

Test infrastructure only (see ``oracle/__init__.py``).
"""
import numpy as np


def lame(E, nu):
    """Lame parameters of an isotropic solid: lambda = E nu / ((1+nu)(1-2nu)),
    mu = E / (2 (1+nu))."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def voigt_d(E, nu):
    """6x6 elasticity matrix C (Eq. (1b)) in Voigt order
    [xx, yy, zz, yz, zx, xy] acting on engineering shear strains."""
    lam, mu = lame(E, nu)
    lam = np.atleast_1d(lam)
    mu = np.atleast_1d(mu)
    D = np.zeros(lam.shape + (6, 6))
    D[..., :3, :3] = lam[..., None, None]
    for i in range(3):
        D[..., i, i] += 2.0 * mu
        D[..., 3 + i, 3 + i] = mu
    return D


def from_wave_speeds(vp, vs, rho):
    """(E, nu) from P- and S-wave speeds and density, as the paper gives its
    layers in Table 3: mu = rho vs^2, lambda = rho vp^2 - 2 mu."""
    mu = rho * vs ** 2
    lam = rho * vp ** 2 - 2.0 * mu
    E = mu * (3.0 * lam + 2.0 * mu) / (lam + mu)
    nu = lam / (2.0 * (lam + mu))
    return E, nu
