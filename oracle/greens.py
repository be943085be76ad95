"""Green's functions of unit fault slips and the regularised slip inversion
(Section 5, Eq. (4) and Eq. (5); the fault loading of Section 2).

Test infrastructure only (see ``oracle/__init__.py``).

Split-node loading (Section 2 cites the split-node technique of Melosh and
Raefsky for the fault).  A node on the fault carries two displacements, one
seen by the elements on each side, with a prescribed jump (the slip)
u+ - u- = s.  Writing u+ = v + s/2 and u- = v - s/2, equilibrium of the pair
gives a problem on the ordinary (unsplit) mesh for the mean field v:

    K v = f,   f = sum_{e on the + side} -K_e s_e / 2 + sum_{e on the - side} K_e s_e / 2,

where s_e is the slip at the element's nodes (zero off the fault).  Away
from the fault the displacement is v itself, which is what a surface
observation sees.

Green's function g_ji: the response at observation DOF j to unit slip basis
function i (Eq. (4): slip = sum_i a_i phi_i).  Inversion (Eq. (5)): the
least-squares solution of [G; alpha L] a = [d; 0], with L a smoothing
matrix and alpha from the L-curve (Hansen): the point of largest curvature
of (log ||G a - d||, log ||L a||) over alpha.
"""
import numpy as np

from .fem import element_stiffness_p2, _dof_map


def split_node_forces(xyz, conn, E, nu, sides, slip):
    """f = sum_e -(side_e / 2) K_e s_e over the elements with side_e = +1 / -1.

    sides (E,) int8, slip (N, 3, n) nodal slips (nonzero at fault nodes only);
    returns f (N, 3, n)."""
    conn = np.asarray(conn)
    N, _, n = slip.shape
    els = np.nonzero(np.asarray(sides) != 0)[0]
    f = np.zeros((3 * N, n))
    if els.size == 0:
        return f.reshape(N, 3, n)
    E = np.broadcast_to(np.asarray(E, dtype=np.float64), (conn.shape[0],))
    nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (conn.shape[0],))
    Ke = element_stiffness_p2(xyz[conn[els]], E[els], nu[els])
    dm = _dof_map(conn[els])
    se = slip.reshape(3 * N, n)[dm]                       # (m, 30, n)
    fe = -(0.5 * np.asarray(sides)[els].astype(np.float64))[:, None, None] * (Ke @ se)
    for r in range(n):
        f[:, r] += np.bincount(dm.ravel(), weights=fe[:, :, r].ravel(), minlength=3 * N)
    return f.reshape(N, 3, n)


def observation_dofs(stations):
    """Flat DOF indices (node * 3 + component) of all components at the stations."""
    st = np.asarray(stations, dtype=np.int64)
    return (3 * st[:, None] + np.arange(3)[None, :]).ravel()


def greens_matrix(solutions, stations):
    """G (3 m, n): the displacement components at the m stations for each of
    the n solved cases (u of shape (N, 3, n))."""
    N, _, n = solutions.shape
    return solutions.reshape(3 * N, n)[observation_dofs(stations)]


def smoothing_matrix(ns, nd, ndir=2):
    """Discrete Laplacian over the (ns x nd) grid of basis functions, per slip
    direction (zero slip assumed beyond the grid): rows 4 a_(i,j) - sum of the
    four neighbours, basis ordered direction-major then (i, j) with j fastest."""
    n1 = ns * nd
    L = np.zeros((ndir * n1, ndir * n1))
    for dct in range(ndir):
        for i in range(ns):
            for j in range(nd):
                row = dct * n1 + i * nd + j
                L[row, row] = 4.0
                for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                    ii, jj = i + di, j + dj
                    if 0 <= ii < ns and 0 <= jj < nd:
                        L[row, dct * n1 + ii * nd + jj] = -1.0
    return L


def regularized_lsq(G, d, L, alpha):
    """a minimising ||G a - d||^2 + alpha^2 ||L a||^2: the least-squares
    solution of the stacked system of Eq. (5) (a library QR least squares)."""
    A = np.vstack([G, alpha * L])
    b = np.concatenate([d, np.zeros(L.shape[0])])
    return np.linalg.lstsq(A, b, rcond=None)[0]


def curvature(x, y, t):
    """Signed curvature of the plane curve (x(t), y(t)) at the samples t,
    derivatives by second-order finite differences."""
    dx, dy = np.gradient(x, t), np.gradient(y, t)
    ddx, ddy = np.gradient(dx, t), np.gradient(dy, t)
    return (dx * ddy - ddx * dy) / (dx * dx + dy * dy) ** 1.5


def l_curve(G, d, L, alphas):
    """Residual norms rho, seminorms eta and solutions over the alphas, and
    the index of the L-curve corner: the largest curvature of
    (log rho, log eta) as a function of log alpha (Hansen's criterion)."""
    alphas = np.asarray(alphas, dtype=np.float64)
    sols = np.stack([regularized_lsq(G, d, L, a) for a in alphas])
    rho = np.linalg.norm(sols @ G.T - d[None, :], axis=1)
    eta = np.linalg.norm(sols @ L.T, axis=1)
    kappa = curvature(np.log(rho), np.log(eta), np.log(alphas))
    return rho, eta, sols, int(np.argmax(kappa)), kappa
