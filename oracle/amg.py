"""The third multigrid level of Algorithm 1: an algebraic coarsening of the
linear (corner) mesh, plain NumPy/SciPy.

Test infrastructure only (see ``oracle/__init__.py``).

The paper coarsens the first-order mesh algebraically (Section 2, "inner loop
level 2"), stores the coarse matrix A2 in 3x3 block compressed rows
(Section 2, EBE paragraph) and maps coarse to fine with P2 (Algorithm 1(a)),
but leaves the coarsening itself to an earlier work.  The reading taken here
is plain aggregation with one 3-DOF (translation) coarse node per aggregate:

* aggregates, in three passes over the corners in increasing id on the
  corner graph (corners joined by an element edge):
    1. a corner whose neighbours are all still free roots a new aggregate made
       of itself and its neighbours;
    2. every corner still free joins the lowest-numbered aggregate among its
       neighbours' pass-1 aggregates;
    3. a corner still free (none can be: a corner left free by pass 1 had an
       aggregated neighbour when it was visited) roots an aggregate with its
       free neighbours.
* the tentative prolongator T maps DOF (I, c) of aggregate I to DOF (a, c)
  of each member a, except where (a, c) is fixed (Dirichlet);
* P2 = (I - omega D1^-1 K1p) T with omega = 2/3 (smoothed aggregation: one
  damped block-Jacobi step applied to T), K1p = K1 with fixed rows and
  columns removed, D1^-1 the level-1 block Jacobi (fixed DOFs: identity);
* A2 = P2^T K1p P2 (Galerkin); a coarse DOF all of whose fine DOFs are fixed
  has an empty row and column and is treated as fixed at level 2.
"""
import numpy as np
import scipy.sparse as sp

from .solve import block_jacobi_inverse


def corner_graph(conn, n_vertices):
    """Neighbour lists of the corner graph (corners joined by a tet edge), increasing."""
    c = np.asarray(conn)[:, :4].astype(np.int64)
    pairs = np.concatenate([c[:, [i, j]] for i in range(4) for j in range(4) if i != j])
    key = np.unique(pairs[:, 0] * n_vertices + pairs[:, 1])
    a, b = key // n_vertices, key % n_vertices
    off = np.searchsorted(a, np.arange(n_vertices + 1))
    return [b[off[v]:off[v + 1]] for v in range(n_vertices)]


def aggregate(nbrs):
    """Aggregate id of every corner (the three passes above); returns (agg, n_agg)."""
    n = len(nbrs)
    agg = np.full(n, -1, dtype=np.int64)
    na = 0
    for v in range(n):  # pass 1
        if agg[v] < 0 and np.all(agg[nbrs[v]] < 0):
            agg[v] = na
            agg[nbrs[v]] = na
            na += 1
    first = agg.copy()
    for v in range(n):  # pass 2
        if first[v] < 0:
            cand = first[nbrs[v]]
            cand = cand[cand >= 0]
            if cand.size:
                agg[v] = cand.min()
    for v in range(n):  # pass 3
        if agg[v] < 0:
            agg[v] = na
            free = nbrs[v][agg[nbrs[v]] < 0]
            agg[free] = na
            na += 1
    return agg, na


OMEGA = 2.0 / 3.0


def prolongation_p2(agg, n_agg, fixed):
    """The tentative prolongator T as a (3 Nv) x (3 Na) 0/1 matrix on DOFs
    (node-major, component-minor); rows of fixed fine DOFs are empty."""
    nv = agg.shape[0]
    fx = np.asarray(fixed).astype(bool)[:nv]
    rows, cols = [], []
    for c in range(3):
        keep = ~fx[:, c]
        v = np.nonzero(keep)[0]
        rows.append(3 * v + c)
        cols.append(3 * agg[v] + c)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(3 * nv, 3 * n_agg))


def coarse_fixed(agg, n_agg, fixed):
    """(Na, 3) bool: coarse DOFs whose fine DOFs are all fixed."""
    fx = np.asarray(fixed).astype(bool)[:agg.shape[0]]
    free = np.zeros((n_agg, 3), dtype=bool)
    for c in range(3):
        np.logical_or.at(free[:, c], agg, ~fx[:, c])
    return ~free


def projected(K1, fixed):
    """K1p = P K1 P: the rows and columns of fixed DOFs removed."""
    keep = sp.diags((~np.asarray(fixed).astype(bool)[:K1.shape[0] // 3]).ravel().astype(float))
    return (keep @ K1 @ keep).tocsr()


def smoothed(T, K1, fixed, omega=OMEGA):
    """P2 = (I - omega D1^-1 K1p) T, D1 the 3x3 diagonal blocks of K1p with the
    fixed DOFs' rows and columns set to identity."""
    nv = K1.shape[0] // 3
    K1p = projected(K1, fixed)
    Dinv = block_jacobi_inverse(K1, np.asarray(fixed)[:nv], nv)
    D = sp.block_diag(list(Dinv)).tocsr()
    return (T - omega * (D @ (K1p @ T))).tocsr()


def galerkin(K1, P2):
    """A2 = P2^T K1 P2."""
    return (P2.T @ K1 @ P2).tocsr()


def level2(conn, n_vertices, K1, fixed, omega=OMEGA):
    """Everything level 2 needs: (agg, n_agg, P2, A2, coarse fixed mask);
    omega = 0 gives the unsmoothed (tentative) prolongator."""
    agg, na = aggregate(corner_graph(conn, n_vertices))
    T = prolongation_p2(agg, na, fixed)
    P2 = smoothed(T, K1, fixed, omega) if omega != 0 else T
    return agg, na, P2, galerkin(projected(K1, fixed), P2), coarse_fixed(agg, na, fixed)
