"""Adjoint gradient of a surface-displacement misfit with respect to the
per-element Young's modulus.

Test infrastructure only (see ``oracle/__init__.py``).

This is an extension beyond the paper, motivated by its inverse analysis
(Section 5, Eq. (5)), where surface responses to many load cases are fitted
to observations.  For L(E) = 1/2 sum_c ||S u_c - d_c||^2 with K(E) u_c = f_c:

    K lambda_c = S^T (S u_c - d_c)          (one extra solve per case; K = K^T)
    dL/dE_e   = - sum_c lambda_{c,e}^T (dK_e/dE_e) u_{c,e},

and since K_e is linear in E_e at fixed Poisson ratio, dK_e/dE_e = K_e / E_e,
i.e. the element stiffness evaluated with E = 1.
"""
import numpy as np

from .fem import assemble, element_stiffness_p2, _dof_map
from .solve import sparse_solve


def misfit(u, S, d):
    """L = 1/2 sum_c ||S u_c - d_c||^2; u (N, 3, n), S flat DOF indices, d (|S|, n)."""
    N, _, n = u.shape
    res = u.reshape(3 * N, n)[S] - d
    return 0.5 * float(np.sum(res * res))


def adjoint_rhs(u, S, d):
    """S^T (S u - d) in the (N, 3, n) layout."""
    N, _, n = u.shape
    out = np.zeros((3 * N, n))
    out[S] = u.reshape(3 * N, n)[S] - d
    return out.reshape(N, 3, n)


def element_gradient(xyz, conn, nu, u, lam, chunk=20000):
    """g_e = - sum_c lambda_{c,e}^T K_e(E=1) u_{c,e}  (E_e-independent form)."""
    conn = np.asarray(conn)
    N, _, n = u.shape
    uf = u.reshape(3 * N, n)
    lf = lam.reshape(3 * N, n)
    nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (conn.shape[0],))
    g = np.zeros(conn.shape[0])
    for s in range(0, conn.shape[0], chunk):
        c = conn[s:s + chunk]
        K1 = element_stiffness_p2(xyz[c], np.ones(c.shape[0]), nu[s:s + chunk])
        dm = _dof_map(c)
        g[s:s + chunk] = -np.einsum("mar,mab,mbr->m", lf[dm], K1, uf[dm])
    return g


def solve_forward(xyz, conn, E, nu, fixed, f):
    K = assemble(xyz, conn, E, nu, n_nodes=xyz.shape[0])
    return sparse_solve(K, f, fixed), K


def loss(xyz, conn, E, nu, fixed, f, S, d):
    u, _ = solve_forward(xyz, conn, E, nu, fixed, f)
    return misfit(u, S, d)


def gradient(xyz, conn, E, nu, fixed, f, S, d):
    """Full adjoint pipeline with direct solves: returns (L, dL/dE, u, lambda)."""
    u, K = solve_forward(xyz, conn, E, nu, fixed, f)
    lam = sparse_solve(K, adjoint_rhs(u, S, d), fixed)
    return misfit(u, S, d), element_gradient(xyz, conn, nu, u, lam), u, lam
