"""Pins of the oracle's adjoint gradient dL/dE_e.

* Central finite differences of the misfit, each evaluated by an independent
  direct solve.
* Euler homogeneity: u(sE) = u(E)/s, so sum_e E_e dL/dE_e = -sum_c (S u_c - d_c) . (S u_c).
* Compliance special case: for C(E) = f^T u the adjoint state is u itself and
  dC/dE_e = -u_e^T (K_e/E_e) u_e; checked against finite differences of C.
"""
import numpy as np

from oracle import adjoint, fem, solve
from paper_1710_08679_amd import meshgen


def setup(nrhs=2):
    m = meshgen.adjoint_mesh(4, 4, 2)
    f, _ = meshgen.dislocation_pair_loads(m, meshgen.rng_for(4, 3), nrhs=nrhs)
    S = meshgen.top_surface_dofs(m)
    d = 1e-2 * meshgen.rng_for(4, 4).standard_normal((S.size, nrhs))
    return m, f, S, d


def test_adjoint_gradient_matches_central_differences():
    m, f, S, d = setup()
    L, g, u, lam = adjoint.gradient(m.xyz, m.conn, m.young, m.poisson, m.fixed, f, S, d)
    rng = np.random.default_rng(11)
    for e in rng.choice(m.n_elem, size=8, replace=False):
        h = 1e-4 * m.young[e]
        Ep = m.young.copy()
        Ep[e] += h
        Em = m.young.copy()
        Em[e] -= h
        fd = (adjoint.loss(m.xyz, m.conn, Ep, m.poisson, m.fixed, f, S, d)
              - adjoint.loss(m.xyz, m.conn, Em, m.poisson, m.fixed, f, S, d)) / (2 * h)
        assert abs(fd - g[e]) <= 1e-5 * abs(g).max()


def test_adjoint_gradient_euler_homogeneity():
    m, f, S, d = setup(nrhs=3)
    L, g, u, lam = adjoint.gradient(m.xyz, m.conn, m.young, m.poisson, m.fixed, f, S, d)
    Su = u.reshape(-1, 3)[S]
    rhs = -np.sum((Su - d) * Su)
    assert abs(np.dot(m.young, g) - rhs) <= 1e-10 * abs(rhs)


def test_compliance_gradient_special_case():
    m, f, S, d = setup(nrhs=1)
    K = fem.assemble(m.xyz, m.conn, m.young, m.poisson)
    u = solve.sparse_solve(K, f, m.fixed)
    g = adjoint.element_gradient(m.xyz, m.conn, m.poisson, u, u)

    def compliance(E):
        Kx = fem.assemble(m.xyz, m.conn, E, m.poisson)
        return float(np.sum(f * solve.sparse_solve(Kx, f, m.fixed)))

    for e in (0, 17, m.n_elem - 1):
        h = 1e-4 * m.young[e]
        Ep = m.young.copy()
        Ep[e] += h
        Em = m.young.copy()
        Em[e] -= h
        fd = (compliance(Ep) - compliance(Em)) / (2 * h)
        assert abs(fd - g[e]) <= 1e-5 * abs(g).max()
    assert np.all(g <= 1e-15 * abs(g).max())  # stiffening never increases compliance
