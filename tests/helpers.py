"""Shared helpers of the GPU parity tests: seeded meshes, oracle references
and the tolerance rule.

Tolerance rule for the EBE products.  Each output entry is a sum of a few
hundred products K_ij x_j formed in the kernel's precision (element geometry
from FP64 coordinates, the rest in the kernel dtype) and accumulated with
atomics in arbitrary order.  Forming K_e from coordinates perturbs it by a
relative amount of order kappa(J_e) u (J_e = the element's edge-vector
matrix, u = unit roundoff), on the oracle's side as on the kernel's, so the
bound is  |y_gpu - y|_i <= c * kappa_max * u * (|K| |x|)_i  with c = 16 for
FP64 and c = 32 for FP32 (the FP32 stress and force steps add a few ulps
more per term); kappa_max is the largest kappa(J_e) of the mesh.
"""
import numpy as np

from oracle import fem
from paper_1710_08679_amd import meshgen

C_TOL = {np.float64: 16.0, np.float32: 32.0}


def unit_roundoff(dtype):
    return float(np.finfo(dtype).eps) / 2.0


def parity_mesh(a=6, b=5, c=4, seed=0, layered=True, bc=False):
    m = meshgen.kuhn_mesh(a, b, c, lengths=(1.2, 1.0, 0.8), jitter=0.2, rng=meshgen.rng_for(77, seed))
    if layered:
        meshgen.set_layers_flat(m)
        m.young = m.young * np.exp(0.3 * meshgen.rng_for(77, 100 + seed).standard_normal(m.n_elem))
    if bc:
        meshgen.fix_faces(m, ((2, 0),))
        m.fixed[meshgen.face_nodes(m, 0, 0), 0] = 1  # a roller: x fixed on x = 0
    return m


def kappa_max(m):
    """Largest 2-norm condition number of the elements' edge-vector matrices."""
    x, c = m.xyz, m.conn
    J = np.stack([x[c[:, 1]] - x[c[:, 0]], x[c[:, 2]] - x[c[:, 0]], x[c[:, 3]] - x[c[:, 0]]], axis=2)
    s = np.linalg.svd(J, compute_uv=False)
    return float(np.max(s[:, 0] / s[:, 2]))


def tol_factor(dtype, kappa):
    return C_TOL[dtype] * kappa * unit_roundoff(dtype)


def assert_close_bound(got, ref, absK, x, dtype, kappa, what=""):
    """|got - ref| <= c kappa u (|K| |x|) elementwise, with ref from the oracle."""
    N, _, n = x.shape
    bound = (absK @ np.abs(x).reshape(3 * N, n)).reshape(got.shape)
    tol = tol_factor(dtype, kappa) * bound + 1e-300
    err = np.abs(got - ref)
    worst = float(np.max(err / tol))
    assert worst <= 1.0, f"{what}: max |err| / bound = {worst:.3g}"
    return worst


def oracle_K(m, order=2):
    n = m.n_nodes if order == 2 else m.n_vertices
    return fem.assemble(m.xyz, m.conn, m.young, m.poisson, order=order, n_nodes=n)


def node_to_elems(conn, nodes):
    """For sampled nodes, the elements that touch them."""
    flat = conn.ravel()
    order = np.argsort(flat, kind="stable")
    sorted_nodes = flat[order]
    out = []
    for v in nodes:
        lo = np.searchsorted(sorted_nodes, v, "left")
        hi = np.searchsorted(sorted_nodes, v, "right")
        out.append(np.unique(order[lo:hi] // conn.shape[1]))
    return out


def sampled_matvec(m, x, nodes):
    """Oracle (K x) and (|K| |x|) at the sampled nodes only, from the element
    matrices of the elements around each node."""
    els = node_to_elems(m.conn, nodes)
    n = x.shape[2]
    y = np.zeros((len(nodes), 3, n))
    b = np.zeros((len(nodes), 3, n))
    for k, (v, es) in enumerate(zip(nodes, els)):
        Ke = fem.element_stiffness_p2(m.xyz[m.conn[es]], m.young[es], m.poisson[es])
        for j, e in enumerate(es):
            a = int(np.nonzero(m.conn[e] == v)[0][0])
            xe = x[m.conn[e]].reshape(30, n)
            rows = Ke[j, 3 * a:3 * a + 3]
            y[k] += rows @ xe
            b[k] += np.abs(rows) @ np.abs(xe)
    return y, b


def restricted_matvec(m, x, nodes):
    """Oracle (K x) and (|K| |x|) at a node set, from the element products of
    every element that touches it (exact there: no other element contributes)."""
    mark = np.zeros(m.n_nodes, dtype=bool)
    mark[nodes] = True
    els = np.nonzero(mark[m.conn].any(axis=1))[0]
    N, _, n = x.shape
    xf = x.reshape(3 * N, n)
    y = np.zeros((3 * N, n))
    b = np.zeros((3 * N, n))
    for s in range(0, els.size, 20000):
        es = els[s:s + 20000]
        Ke = fem.element_stiffness_p2(m.xyz[m.conn[es]], m.young[es], m.poisson[es])
        dm = (3 * m.conn[es][:, :, None].astype(np.int64) + np.arange(3)).reshape(es.size, 30)
        xe = xf[dm]
        ye = Ke @ xe
        be = np.abs(Ke) @ np.abs(xe)
        for r in range(n):
            y[:, r] += np.bincount(dm.ravel(), weights=ye[:, :, r].ravel(), minlength=3 * N)
            b[:, r] += np.bincount(dm.ravel(), weights=be[:, :, r].ravel(), minlength=3 * N)
    return y.reshape(N, 3, n)[nodes], b.reshape(N, 3, n)[nodes]
