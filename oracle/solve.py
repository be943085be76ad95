"""Reference solves of K u = f (Section 2, Eq. (2)) with homogeneous or
prescribed Dirichlet DOFs.

Test infrastructure only (see ``oracle/__init__.py``).

The converged solution of Eq. (2) has a plain definition, u_f = K_ff^-1
(f_f - K_fb u_b), so the references here are direct solves (dense Cholesky
or sparse LU, both library routines) plus a textbook preconditioned CG used
where a direct factorisation does not fit.  Vectors use the (N, 3, n)
layout, RHS index fastest.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def free_dofs(fixed):
    return np.nonzero(~np.asarray(fixed).astype(bool).ravel())[0]


def _split(K, fixed, f, u_fixed):
    N = f.shape[0]
    n = f.shape[2]
    fr = free_dofs(fixed)
    fx = np.nonzero(np.asarray(fixed).astype(bool).ravel())[0]
    Kc = K.tocsr()
    Kff = Kc[fr][:, fr]
    rhs = f.reshape(3 * N, n)[fr]
    if u_fixed is not None and fx.size:
        ub = np.asarray(u_fixed, dtype=np.float64).reshape(3 * N, -1)[fx]
        rhs = rhs - Kc[fr][:, fx] @ ub
    return Kff, rhs, fr, fx


def _scatter(sol, N, n, fr, fx, u_fixed):
    u = np.zeros((3 * N, n))
    u[fr] = sol
    if u_fixed is not None and fx.size:
        u[fx] = np.asarray(u_fixed, dtype=np.float64).reshape(3 * N, -1)[fx]
    return u.reshape(N, 3, n)


def dense_solve(K, f, fixed, u_fixed=None):
    """Dense Cholesky of K_ff (meshes up to ~1e4 DOF)."""
    f = np.asarray(f, dtype=np.float64)
    N, _, n = f.shape
    Kff, rhs, fr, fx = _split(K, fixed, f, u_fixed)
    c = sla.cho_factor(Kff.toarray(), lower=True)
    return _scatter(sla.cho_solve(c, rhs), N, n, fr, fx, u_fixed)


def sparse_solve(K, f, fixed, u_fixed=None):
    """Sparse LU (SuperLU) of K_ff, for meshes up to a few 1e5 DOF."""
    f = np.asarray(f, dtype=np.float64)
    N, _, n = f.shape
    Kff, rhs, fr, fx = _split(K, fixed, f, u_fixed)
    lu = spla.splu(sp.csc_matrix(Kff))
    return _scatter(lu.solve(rhs), N, n, fr, fx, u_fixed)


def block_jacobi_inverse(K, fixed, n_nodes):
    """Inverted 3x3 nodal diagonal blocks of P_f K P_f, with fixed rows and
    columns replaced by identity (Algorithm 1, 'diag[K]')."""
    Kc = K.tocsr()
    idx = np.arange(n_nodes) * 3
    blk = np.zeros((n_nodes, 3, 3))
    for a in range(3):
        for b in range(3):
            blk[:, a, b] = np.asarray(Kc[idx + a, idx + b]).ravel()
    fx = np.asarray(fixed).astype(bool)
    for a in range(3):
        blk[fx[:, a], a, :] = 0.0
        blk[fx[:, a], :, a] = 0.0
        blk[fx[:, a], a, a] = 1.0
    return np.linalg.inv(blk)


def residual(K, u, f, fixed):
    """(N, 3, n) residual P_f (f - K u)."""
    N, _, n = u.shape
    r = f.reshape(3 * N, n) - K @ u.reshape(3 * N, n)
    r = r.reshape(N, 3, n)
    r[np.asarray(fixed).astype(bool)] = 0.0
    return r


def pcg(K, f, fixed, tol=1e-13, maxit=100000, u0=None):
    """Textbook CG with 3x3 block-Jacobi preconditioning on P_f K P_f, FP64,
    one column at a time.  Stops when ||r_j|| / ||f_j|| <= tol.

    Returns (u, iterations per column).
    """
    f = np.asarray(f, dtype=np.float64)
    N, _, n = f.shape
    fx = np.asarray(fixed).astype(bool)
    Minv = block_jacobi_inverse(K, fixed, N)
    Kc = K.tocsr()

    def A(v):
        w = np.array(v)
        w[fx] = 0.0
        y = (Kc @ w.reshape(-1)).reshape(N, 3)
        y[fx] = 0.0
        return y

    u = np.zeros((N, 3, n)) if u0 is None else np.array(u0, dtype=np.float64)
    its = []
    for j in range(n):
        b = f[:, :, j].copy()
        b[fx] = 0.0
        x = u[:, :, j].copy()
        x[fx] = 0.0
        r = b - A(x)
        nb = np.linalg.norm(b)
        if nb == 0.0:
            u[:, :, j] = 0.0
            its.append(0)
            continue
        z = np.einsum("nab,nb->na", Minv, r)
        p = z.copy()
        rz = np.vdot(r, z)
        k = 0
        while np.linalg.norm(r) / nb > tol and k < maxit:
            q = A(p)
            alpha = rz / np.vdot(p, q)
            x += alpha * p
            r -= alpha * q
            z = np.einsum("nab,nb->na", Minv, r)
            rz_new = np.vdot(r, z)
            p = z + (rz_new / rz) * p
            rz = rz_new
            k += 1
        u[:, :, j] = x
        its.append(k)
    return u, its
