"""Element stiffness, global assembly and the EBE product by definition.

Test infrastructure only (see ``oracle/__init__.py``).

* Section 2, Eq. (1a-c): small-strain isotropic linear elasticity.
* Section 2, Eq. (2): second-order (10-node) tetrahedral discretisation K u = f.
* Section 2, Eq. (3): f = sum_i Q_i K_i Q_i^T u, with K_i the element stiffness
  and Q_i the local-to-global node map.

Textbook isoparametric formulation: K_e = int B^T D B dV, evaluated with
the 4-point degree-2 tetrahedron rule at each point's own Jacobian.  For a
straight-sided element the integrand is a quadratic polynomial and the rule
is exact.  Local node order: vertices 0..3, then edges (0,1), (1,2), (0,2),
(0,3), (1,3), (2,3).
"""
import numpy as np
import scipy.sparse as sp

from .material import voigt_d

EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))


def barycentric(xi):
    """xi (..., 3) reference coordinates -> L (..., 4) with L0 = 1 - sum(xi)."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.concatenate([1.0 - xi.sum(axis=-1, keepdims=True), xi], axis=-1)


# dL_i / dxi_d for the four barycentric coordinates
_DL = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def p2_shape(xi):
    """Quadratic Lagrange shape functions on the reference tetrahedron.

    Returns N (..., 10) and dN/dxi (..., 10, 3).  Vertex i: L_i (2 L_i - 1);
    edge (i, j): 4 L_i L_j.
    """
    L = barycentric(xi)
    shp = L.shape[:-1]
    N = np.empty(shp + (10,))
    dN = np.empty(shp + (10, 3))
    for i in range(4):
        N[..., i] = L[..., i] * (2.0 * L[..., i] - 1.0)
        dN[..., i, :] = (4.0 * L[..., i] - 1.0)[..., None] * _DL[i]
    for k, (i, j) in enumerate(EDGES):
        N[..., 4 + k] = 4.0 * L[..., i] * L[..., j]
        dN[..., 4 + k, :] = 4.0 * (L[..., j][..., None] * _DL[i] + L[..., i][..., None] * _DL[j])
    return N, dN


def p1_shape(xi):
    """Linear shape functions N_i = L_i; returns N (..., 4), dN/dxi (..., 4, 3)."""
    L = barycentric(xi)
    return L, np.broadcast_to(_DL, L.shape[:-1] + (4, 3)).copy()


def tet_rule_4():
    """Symmetric 4-point rule, exact for polynomials of degree 2.

    Points: barycentric (a, b, b, b) and permutations with
    a = (5 + 3 sqrt 5) / 20, b = (5 - sqrt 5) / 20; each weight is 1/4 of the
    reference volume 1/6.
    """
    a = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
    b = (5.0 - np.sqrt(5.0)) / 20.0
    bary = np.array([[a, b, b, b], [b, a, b, b], [b, b, a, b], [b, b, b, a]])
    return bary[:, 1:], np.full(4, 1.0 / 24.0)


def strain_matrix(dNdx):
    """B (..., 6, 3n) mapping nodal displacements to engineering strains
    [e_xx, e_yy, e_zz, g_yz, g_zx, g_xy] (Eq. (1a))."""
    n = dNdx.shape[-2]
    B = np.zeros(dNdx.shape[:-2] + (6, 3 * n))
    gx, gy, gz = dNdx[..., 0], dNdx[..., 1], dNdx[..., 2]
    B[..., 0, 0::3] = gx
    B[..., 1, 1::3] = gy
    B[..., 2, 2::3] = gz
    B[..., 3, 1::3] = gz
    B[..., 3, 2::3] = gy
    B[..., 4, 0::3] = gz
    B[..., 4, 2::3] = gx
    B[..., 5, 0::3] = gy
    B[..., 5, 1::3] = gx
    return B


def _stiffness(xe, E, nu, shape_fn, rule):
    """Generic isoparametric stiffness: xe (m, n, 3) node coords, E/nu (m,)."""
    xe = np.asarray(xe, dtype=np.float64)
    m, n, _ = xe.shape
    D = voigt_d(np.broadcast_to(E, (m,)), np.broadcast_to(nu, (m,)))  # (m, 6, 6)
    pts, wts = rule
    K = np.zeros((m, 3 * n, 3 * n))
    for q in range(len(wts)):
        _, dN = shape_fn(pts[q])                       # (n, 3) dN/dxi
        J = np.einsum("man,kn->mak", xe.transpose(0, 2, 1), dN.T)  # J[c, d] = dx_c/dxi_d
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)                        # Jinv[d, c] = dxi_d/dx_c
        dNdx = np.einsum("nd,mdc->mnc", dN, Jinv)      # (m, n, 3)
        B = strain_matrix(dNdx)                        # (m, 6, 3n)
        K += (wts[q] * np.abs(detJ))[:, None, None] * (B.transpose(0, 2, 1) @ (D @ B))  # B^T D B
    return K


def element_stiffness_p2(xe, E, nu, rule=None):
    """(m, 30, 30) stiffness of 10-node tetrahedra (Eq. (2)); DOF order node-major (x, y, z)."""
    return _stiffness(xe, E, nu, p2_shape, tet_rule_4() if rule is None else rule)


def element_stiffness_p1(xe, E, nu):
    """(m, 12, 12) stiffness of 4-node tetrahedra (the coarse level; constant strain, 1 point)."""
    return _stiffness(xe, E, nu, p1_shape, (np.array([[0.25, 0.25, 0.25]]), np.array([1.0 / 6.0])))


def _dof_map(conn):
    return (3 * conn[:, :, None].astype(np.int64) + np.arange(3)[None, None, :]).reshape(conn.shape[0], -1)


def assemble(xyz, conn, E, nu, order=2, n_nodes=None, chunk=20000):
    """Global stiffness K = sum_i Q_i K_i Q_i^T (Eq. (3)) as scipy CSR.

    order=2: 10-node elements on all nodes; order=1: 4-node elements on the
    corner nodes (conn[:, :4]); n_nodes sets the matrix size (3 n_nodes).
    """
    conn = np.asarray(conn)
    if order == 1:
        conn = conn[:, :4]
    if n_nodes is None:
        n_nodes = int(conn.max()) + 1
    ndof = 3 * n_nodes
    K = sp.csr_matrix((ndof, ndof))
    E = np.broadcast_to(np.asarray(E, dtype=np.float64), (conn.shape[0],))
    nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (conn.shape[0],))
    kfun = element_stiffness_p2 if order == 2 else element_stiffness_p1
    for s in range(0, conn.shape[0], chunk):
        c = conn[s:s + chunk]
        Ke = kfun(xyz[c], E[s:s + chunk], nu[s:s + chunk])
        dm = _dof_map(c)
        nd = dm.shape[1]
        rows = np.repeat(dm, nd, axis=1).ravel()
        cols = np.tile(dm, (1, nd)).ravel()
        K = K + sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(ndof, ndof)).tocsr()
    K.sum_duplicates()
    return K


def ebe_apply(xyz, conn, E, nu, x, order=2, chunk=20000):
    """EBE product by definition (Eq. (3)): y = sum_i Q_i K_i Q_i^T x.

    x has layout (N, 3, n) (RHS index fastest, as in the multi-vector form of
    Section 3.1); returns y with the same layout.  Element matrices are formed
    densely by quadrature; nothing is cached.
    """
    conn = np.asarray(conn)
    if order == 1:
        conn = conn[:, :4]
    x = np.asarray(x, dtype=np.float64)
    N, _, n = x.shape
    xf = x.reshape(3 * N, n)
    y = np.zeros((3 * N, n))
    E = np.broadcast_to(np.asarray(E, dtype=np.float64), (conn.shape[0],))
    nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (conn.shape[0],))
    kfun = element_stiffness_p2 if order == 2 else element_stiffness_p1
    for s in range(0, conn.shape[0], chunk):
        c = conn[s:s + chunk]
        Ke = kfun(xyz[c], E[s:s + chunk], nu[s:s + chunk])
        dm = _dof_map(c)
        ye = Ke @ xf[dm]                                  # K_i (Q_i^T x), element by element
        for r in range(n):
            y[:, r] += np.bincount(dm.ravel(), weights=ye[:, :, r].ravel(), minlength=3 * N)
    return y.reshape(N, 3, n)


def mask_fixed(v, fixed):
    """Zero the fixed DOFs of a (N, 3, n) array (the projection P_f)."""
    out = np.array(v, dtype=np.float64, copy=True)
    out[np.asarray(fixed).astype(bool)] = 0.0
    return out


def matvec_bc(K, x, fixed):
    """y = P_f K P_f x for x of layout (N, 3, n), with K a global CSR matrix."""
    N, _, n = x.shape
    y = K @ mask_fixed(x, fixed).reshape(3 * N, n)
    return mask_fixed(y.reshape(N, 3, n), fixed)


def diag_blocks(K, n_nodes):
    """(N, 3, 3) nodal diagonal blocks of a global matrix (the 3x3 block Jacobi of
    Algorithm 1, 'diag[ ]')."""
    out = np.zeros((n_nodes, 3, 3))
    Kc = K.tocsr()
    for a in range(3):
        for b in range(3):
            out[:, a, b] = np.asarray(Kc[np.arange(n_nodes) * 3 + a, np.arange(n_nodes) * 3 + b]).ravel()
    return out


def prolongation_p1(conn, n_nodes, n_vertices):
    """Scalar P_1 (n_nodes x n_vertices): the same mesh without edge nodes
    (Section 2, multigrid): a vertex keeps its value, an edge node takes the
    mean of its two end vertices (exact for linear fields)."""
    conn = np.asarray(conn)
    rows = [np.arange(n_vertices)]
    cols = [np.arange(n_vertices)]
    vals = [np.ones(n_vertices)]
    for k, (i, j) in enumerate(EDGES):
        e = conn[:, 4 + k]
        for v in (conn[:, i], conn[:, j]):
            rows.append(e)
            cols.append(v)
            vals.append(np.full(e.size, 0.5))
    rows = np.concatenate(rows).astype(np.int64)
    cols = np.concatenate(cols).astype(np.int64)
    vals = np.concatenate(vals)
    # an edge node appears in every element around its edge: keep one entry per (row, col)
    _, first = np.unique(rows * n_vertices + cols, return_index=True)
    return sp.csr_matrix((vals[first], (rows[first], cols[first])), shape=(n_nodes, n_vertices))


def apply_scalar_op(P, v):
    """Apply a scalar node operator to each component / column of (M, 3, n)."""
    M, _, n = v.shape
    out = P @ v.reshape(M, 3 * n)
    return out.reshape(P.shape[0], 3, n)
