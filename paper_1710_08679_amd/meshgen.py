"""Seeded synthetic inputs for the multi-case EBE solver.

Builds Kuhn-split hexahedral lattices of straight-sided 10-node tetrahedra,
layered crust-like materials, nodal loads and per-DOF Dirichlet masks.  The
shapes follow the paper's workloads (Section 4, Tables 3 and 5): about four
DOF per element, layered elastic moduli, a few million DOF per GPU.

This module only *builds inputs*.  It contains none of the solver's
arithmetic (no shape functions, no stiffness, no products) and is shared by
the GPU path's tests/benchmarks and by the CPU oracle's tests; neither side
imports the other.

Conventions
-----------
* Local node order of a 10-node tetrahedron: vertices 0..3, then the edge
  nodes of edges (0,1), (1,2), (0,2), (0,3), (1,3), (2,3).
* Orientation: det[x1-x0, x2-x0, x3-x0] > 0.
* Numbering is vertex-first: nodes 0..n_vertices-1 are tetrahedron corners,
  the rest are edge (mid-side) nodes.  Within each group nodes are numbered
  in order of first touch while walking elements, and elements walk hexes in
  Morton order, so a contiguous range of elements touches a compact node set.
* Seeds: ``numpy.random.default_rng(SeedSequence([1710, 8679, cfg, item]))``.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

VTK_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))


def rng_for(cfg: int, item: int) -> np.random.Generator:
    """Seeded generator for workload ``cfg`` and stream ``item``."""
    return np.random.default_rng(np.random.SeedSequence([1710, 8679, int(cfg), int(item)]))


def _part1by2(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton3(i, j, k) -> np.ndarray:
    """3-D Morton (Z-order) code of integer lattice indices."""
    return _part1by2(np.asarray(i)) | (_part1by2(np.asarray(j)) << np.uint64(1)) | (
        _part1by2(np.asarray(k)) << np.uint64(2))


@dataclass
class Mesh:
    """A mesh of 10-node tetrahedra plus per-element material (straight-sided
    as built; ``quadratic_map`` and ``curve_edges`` curve them)."""
    xyz: np.ndarray            # (N, 3) float64 node coordinates
    conn: np.ndarray           # (E, 10) int32 connectivity, VTK local order
    n_vertices: int            # nodes [0, n_vertices) are corners
    young: np.ndarray          # (E,) float64 Young's modulus
    poisson: np.ndarray        # (E,) float64 Poisson ratio
    fixed: np.ndarray          # (N, 3) uint8, 1 = Dirichlet-fixed DOF
    grid: tuple = (0, 0, 0)    # hexes per axis
    lengths: tuple = (1.0, 1.0, 1.0)
    refined: np.ndarray = field(default=None, repr=False)  # (N, 3) int32 lattice coords (half-h units)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_dof(self) -> int:
        return 3 * self.n_nodes

    @property
    def h(self) -> np.ndarray:
        return np.asarray(self.lengths, dtype=np.float64) / np.asarray(self.grid, dtype=np.float64)

    def edge_endpoints(self) -> np.ndarray:
        """(N - n_vertices, 2) int32: the two corner nodes of every edge node."""
        out = np.full((self.n_nodes - self.n_vertices, 2), -1, dtype=np.int32)
        for k, (p, q) in enumerate(VTK_EDGES):
            out[self.conn[:, 4 + k] - self.n_vertices, 0] = self.conn[:, p]
            out[self.conn[:, 4 + k] - self.n_vertices, 1] = self.conn[:, q]
        return out

    def centroids(self) -> np.ndarray:
        return self.xyz[self.conn[:, :4]].mean(axis=1)


def kuhn_mesh(a: int, b: int, c: int, lengths=(1.0, 1.0, 1.0), jitter: float = 0.0,
              rng: np.random.Generator | None = None) -> Mesh:
    """a x b x c hexes on [0,Lx]x[0,Ly]x[0,Lz], each split into 6 tetrahedra
    sharing the hex main diagonal (Kuhn/Freudenthal split, conforming).

    ``jitter`` moves interior corner nodes by U(-jitter, jitter)*h per axis;
    edge nodes are then put back at edge midpoints so elements stay straight.
    Material defaults to E=1, nu=0.25; no DOF is fixed.
    """
    a, b, c = int(a), int(b), int(c)
    nx, ny, nz = 2 * a + 1, 2 * b + 1, 2 * c + 1
    ii, jj, kk = np.meshgrid(np.arange(a), np.arange(b), np.arange(c), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    order = np.argsort(morton3(ii, jj, kk), kind="stable")
    base = 2 * np.stack([ii[order], jj[order], kk[order]], axis=1).astype(np.int32)  # (H, 3)

    eye = np.eye(3, dtype=np.int32)
    corner_off = []
    for perm in itertools.permutations(range(3)):
        o1 = 2 * eye[perm[0]]
        o2 = o1 + 2 * eye[perm[1]]
        o3 = np.array([2, 2, 2], dtype=np.int32)
        inv = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
        if inv % 2 == 1:  # odd permutation: negative volume, swap corners 1 and 2
            o1, o2 = o2, o1
        corner_off.append(np.stack([np.zeros(3, np.int32), o1, o2, o3]))
    corner_off = np.stack(corner_off)  # (6, 4, 3)

    H = base.shape[0]
    corners = (base[:, None, None, :] + corner_off[None]).reshape(H * 6, 4, 3)
    edges = np.stack([(corners[:, p] + corners[:, q]) // 2 for p, q in VTK_EDGES], axis=1)
    R = np.concatenate([corners, edges], axis=1)  # (E, 10, 3) refined lattice coords
    del corners, edges
    lin = (R[..., 0].astype(np.int64) + nx * (R[..., 1].astype(np.int64) + ny * R[..., 2].astype(np.int64)))

    newid = np.full(nx * ny * nz, -1, dtype=np.int64)
    uq, first = np.unique(lin[:, :4].ravel(), return_index=True)
    uq = uq[np.argsort(first, kind="stable")]
    nv = uq.size
    newid[uq] = np.arange(nv)
    ue, first = np.unique(lin[:, 4:].ravel(), return_index=True)
    ue = ue[np.argsort(first, kind="stable")]
    newid[ue] = nv + np.arange(ue.size)
    n_nodes = nv + ue.size
    conn = newid[lin].astype(np.int32)
    del lin

    refined = np.empty((n_nodes, 3), dtype=np.int32)
    refined[conn.ravel()] = R.reshape(-1, 3)
    del R
    h = np.asarray(lengths, dtype=np.float64) / np.array([a, b, c], dtype=np.float64)
    xyz = refined.astype(np.float64) * (0.5 * h)
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs a seeded rng")
        rv = refined[:nv]
        interior = np.all((rv > 0) & (rv < np.array([2 * a, 2 * b, 2 * c])), axis=1)
        d = rng.uniform(-jitter, jitter, size=(nv, 3)) * h
        xyz[:nv][interior] += d[interior]
        for k, (p, q) in enumerate(VTK_EDGES):
            xyz[conn[:, 4 + k]] = 0.5 * (xyz[conn[:, p]] + xyz[conn[:, q]])
    E = conn.shape[0]
    return Mesh(xyz=xyz, conn=conn, n_vertices=int(nv), young=np.ones(E), poisson=np.full(E, 0.25),
                fixed=np.zeros((n_nodes, 3), dtype=np.uint8), grid=(a, b, c),
                lengths=tuple(float(x) for x in lengths), refined=refined)


# --------------------------------------------------------------------------
# materials
# --------------------------------------------------------------------------
LAYER_TRIPLET = ((1.0, 0.25), (3.0, 0.27), (8.0, 0.30))  # top -> bottom (E, nu)


def set_layers_flat(mesh: Mesh, z_cuts=(2.0 / 3.0, 1.0 / 3.0), layers=LAYER_TRIPLET) -> None:
    """Horizontal layers by element-centroid z: z >= z_cuts[0] is layers[0], ..."""
    zc = mesh.centroids()[:, 2] / mesh.lengths[2]
    idx = np.full(mesh.n_elem, len(layers) - 1, dtype=np.int64)
    for li in range(len(z_cuts) - 1, -1, -1):
        idx[zc >= z_cuts[li]] = li
    E = np.array([l[0] for l in layers])
    nu = np.array([l[1] for l in layers])
    mesh.young, mesh.poisson = E[idx].copy(), nu[idx].copy()


def sinusoidal_interfaces(rng: np.random.Generator, levels=(0.7, 0.35), period=2.0):
    """Seeded interface depth functions z_i(x, y) = level_i + A sin(.) sin(.)."""
    out = []
    for lev in levels:
        A = rng.uniform(0.02, 0.08)
        k, m = rng.integers(1, 3, size=2)
        ph, ps = rng.uniform(0.0, 2.0 * np.pi, size=2)
        out.append((float(lev), float(A), int(k), int(m), float(ph), float(ps)))

    def depth(i, x, y):
        lev, A, k, m, ph, ps = out[i]
        return lev + A * np.sin(2 * np.pi * k * x / period + ph) * np.sin(2 * np.pi * m * y / period + ps)
    return depth, out


def set_layers_sinusoidal(mesh: Mesh, rng: np.random.Generator, layers=LAYER_TRIPLET) -> list:
    depth, params = sinusoidal_interfaces(rng)
    cen = mesh.centroids()
    z1 = depth(0, cen[:, 0], cen[:, 1])
    z2 = depth(1, cen[:, 0], cen[:, 1])
    idx = np.where(cen[:, 2] >= z1, 0, np.where(cen[:, 2] >= z2, 1, 2))
    E = np.array([l[0] for l in layers])
    nu = np.array([l[1] for l in layers])
    mesh.young, mesh.poisson = E[idx].copy(), nu[idx].copy()
    return params


# Table 3 of the paper: (Vp [m/s], Vs [m/s], rho [kg/m^3]) of the two layers.
PAPER_TABLE3 = ((1600.0, 400.0, 1850.0), (5800.0, 3000.0, 2700.0))


# --------------------------------------------------------------------------
# boundary masks and loads
# --------------------------------------------------------------------------
def face_nodes(mesh: Mesh, axis: int, side: int) -> np.ndarray:
    """Node ids on a domain face (axis 0/1/2, side 0 = min, 1 = max)."""
    lim = 0 if side == 0 else 2 * mesh.grid[axis]
    return np.nonzero(mesh.refined[:, axis] == lim)[0]


def fix_faces(mesh: Mesh, faces) -> None:
    """Fix all three DOFs of the nodes on the given (axis, side) faces."""
    for axis, side in faces:
        mesh.fixed[face_nodes(mesh, axis, side), :] = 1


BOX_SIDES_AND_BOTTOM = ((2, 0), (0, 0), (0, 1), (1, 0), (1, 1))


def top_face_random_loads(mesh: Mesh, rng: np.random.Generator, nrhs: int = 1) -> np.ndarray:
    """(N, 3, nrhs) nodal loads: each component of each top-face node ~ U(-1, 1)."""
    f = np.zeros((mesh.n_nodes, 3, nrhs))
    top = face_nodes(mesh, 2, 1)
    f[top] = rng.uniform(-1.0, 1.0, size=(top.size, 3, nrhs))
    f[mesh.fixed.astype(bool)] = 0.0
    return f


def dislocation_pair_loads(mesh: Mesh, rng: np.random.Generator, nrhs: int = 16,
                           center=(1.0, 1.0, 0.5), dip_deg: float = 30.0, half_extent: float = 0.3):
    """(N, 3, nrhs) zero-net-force body-force pairs on a dipping plane.

    Case j: a seeded point p on a plane striking along x and dipping
    ``dip_deg`` through ``center``; slip direction alternates dip / strike.
    +s goes on the node nearest p + h n, -s on the node nearest p - h n.
    """
    strike = np.array([1.0, 0.0, 0.0])
    dip = np.deg2rad(dip_deg)
    ddir = np.array([0.0, np.cos(dip), -np.sin(dip)])
    normal = np.cross(strike, ddir)
    h = float(mesh.h.min())
    f = np.zeros((mesh.n_nodes, 3, nrhs))
    free = ~mesh.fixed.astype(bool).any(axis=1)
    cand = np.nonzero(free)[0]
    pts = mesh.xyz[cand]
    info = []
    for j in range(nrhs):
        s_, d_ = rng.uniform(-half_extent, half_extent, size=2)
        p = np.asarray(center) + s_ * strike + d_ * ddir
        slip = ddir if j % 2 == 0 else strike
        a = cand[np.argmin(((pts - (p + h * normal)) ** 2).sum(axis=1))]
        bnode = cand[np.argmin(((pts - (p - h * normal)) ** 2).sum(axis=1))]
        f[a, :, j] += slip
        f[bnode, :, j] -= slip
        info.append((p, a, bnode))
    return f, info


def lognormal_material(mesh: Mesh, rng: np.random.Generator, sigma: float = 0.3) -> None:
    """E_e <- E_e * exp(sigma * xi_e), xi_e ~ N(0, 1)."""
    mesh.young = mesh.young * np.exp(sigma * rng.standard_normal(mesh.n_elem))


def shuffled(mesh: Mesh, rng: np.random.Generator) -> Mesh:
    """The same mesh with its elements in random order and its node ids
    permuted at random within the corners and within the edge nodes (so the
    numbering stays vertex-first): the unordered numbering of a general
    unstructured mesh, where consecutive elements share few nodes."""
    pe = rng.permutation(mesh.n_elem)
    nv = mesh.n_vertices
    newid = np.concatenate([rng.permutation(nv), nv + rng.permutation(mesh.n_nodes - nv)])  # old -> new
    xyz = np.empty_like(mesh.xyz)
    xyz[newid] = mesh.xyz
    fixed = np.empty_like(mesh.fixed)
    fixed[newid] = mesh.fixed
    refined = None
    if mesh.refined is not None:
        refined = np.empty_like(mesh.refined)
        refined[newid] = mesh.refined
    return Mesh(xyz=xyz, conn=newid[mesh.conn[pe]].astype(np.int32), n_vertices=nv, young=mesh.young[pe].copy(),
                poisson=mesh.poisson[pe].copy(), fixed=fixed, grid=mesh.grid, lengths=mesh.lengths,
                refined=refined)


def _with_xyz(mesh: Mesh, xyz: np.ndarray) -> Mesh:
    return Mesh(xyz=xyz, conn=mesh.conn.copy(), n_vertices=mesh.n_vertices, young=mesh.young.copy(),
                poisson=mesh.poisson.copy(), fixed=mesh.fixed.copy(), grid=mesh.grid, lengths=mesh.lengths,
                refined=None if mesh.refined is None else mesh.refined.copy())


def quadratic_map(mesh: Mesh, c: float) -> Mesh:
    """The mesh with every node (corners and edge nodes) moved by the global
    map x -> (x + c x^2, y, z).  Edge nodes leave their edge midpoints, so
    the elements become curved; a quadratic element reproduces the mapped
    geometry exactly (its interpolation of a quadratic map is the map)."""
    xyz = mesh.xyz.copy()
    xyz[:, 0] = xyz[:, 0] + c * xyz[:, 0] ** 2
    return _with_xyz(mesh, xyz)


def curve_edges(mesh: Mesh, rng: np.random.Generator, amp: float = 0.05) -> Mesh:
    """The mesh with each edge node moved off its edge midpoint by a seeded
    random vector of length at most amp times that edge's length (corners
    stay): curved tetrahedra of a general shape."""
    ends = mesh.edge_endpoints()
    ln = np.linalg.norm(mesh.xyz[ends[:, 1]] - mesh.xyz[ends[:, 0]], axis=1)
    d = rng.uniform(-1.0, 1.0, size=(ends.shape[0], 3)) / np.sqrt(3.0)
    xyz = mesh.xyz.copy()
    xyz[mesh.n_vertices:] += amp * ln[:, None] * d
    return _with_xyz(mesh, xyz)


def hub_mesh(arms: int) -> Mesh:
    """A hub corner c shared by `arms` arms of two tetrahedra each: arm i is
    (c, a_i, b_i, d_i) and (a_i, b_i, d_i, t_i), rotated by 2 pi i / arms
    about the z axis (arms overlap in space: only the operator matters), with
    a_i, b_i and t_i fully fixed.  Corner ids: t_i first, then a_i, b_i, d_i,
    then c, so every t_i roots its own aggregate when the corner graph is
    coarsened in increasing id and c couples all of them: a coarse operator
    whose rows couple `arms` aggregates."""
    M = int(arms)
    t = np.arange(M)
    a, b, d = M + 3 * t, M + 3 * t + 1, M + 3 * t + 2
    c = 4 * M
    nv = 4 * M + 1
    e0 = nv + 9 * t  # 9 edge nodes per arm: ca, ab, cb, cd, ad, bd, at, bt, dt
    ca, ab, cb, cd, ad, bd, at, bt, dt = (e0 + k for k in range(9))
    conn = np.concatenate([
        np.stack([np.full(M, c), a, b, d, ca, ab, cb, cd, ad, bd], axis=1),
        np.stack([a, b, d, t, ab, bd, ad, at, bt, dt], axis=1)]).astype(np.int32)
    n = nv + 9 * M
    xyz = np.zeros((n, 3))
    th = 2.0 * np.pi * t / M
    cs, sn = np.cos(th), np.sin(th)

    def rot(p):
        return np.stack([cs * p[0] - sn * p[1], sn * p[0] + cs * p[1], np.full(M, float(p[2]))], axis=1)

    xyz[a], xyz[b], xyz[d], xyz[t] = rot((1.0, 0.0, 0.0)), rot((0.0, 1.0, 0.0)), rot((0.0, 0.0, 1.0)), \
        rot((1.0, 1.0, 1.0))
    for k, (p, q) in enumerate(((c, a), (a, b), (c, b), (c, d), (a, d), (b, d), (a, t), (b, t), (d, t))):
        xyz[e0 + k] = 0.5 * (xyz[p] + xyz[q])
    fixed = np.zeros((n, 3), dtype=np.uint8)
    fixed[np.concatenate([a, b, t])] = 1
    E = conn.shape[0]
    return Mesh(xyz=xyz, conn=conn, n_vertices=nv, young=np.ones(E), poisson=np.full(E, 0.25), fixed=fixed)


# --------------------------------------------------------------------------
# a fault for unit-slip loading, and surface observation stations
# --------------------------------------------------------------------------
@dataclass
class Fault:
    """A planar fault patch made of element faces: the plane y - z = c of a
    Kuhn lattice (refined coordinates r_y - r_z = k, k even), dipping 45
    degrees, striking along x, with unit slip basis functions on it.

    nodes    fault-patch node ids (on the plane, inside the patch rectangle)
    coords   (n_fault, 2) in-plane coordinates (x, eta), eta = (y + z) / sqrt 2
    sides    (E,) int8: +1 / -1 for elements touching a fault-patch node on
             the side y - z > c / y - z < c, 0 for the others
    basis    (n_fault, n_basis) basis values at the fault nodes
    dirs     (n_basis, 3) slip direction (unit vector) of each basis function
    """
    k: int
    normal: np.ndarray
    strike: np.ndarray
    dip: np.ndarray
    nodes: np.ndarray
    coords: np.ndarray
    sides: np.ndarray
    basis: np.ndarray
    dirs: np.ndarray
    knots: tuple

    @property
    def n_basis(self) -> int:
        return int(self.basis.shape[1])

    def slip(self, n_nodes: int, cols) -> np.ndarray:
        """(n_nodes, 3, len(cols)) nodal slip vectors of the chosen basis
        functions: B_i(x, eta) times the slip direction at fault nodes, zero
        elsewhere."""
        cols = np.asarray(cols)
        out = np.zeros((n_nodes, 3, cols.size))
        out[self.nodes] = self.basis[:, None, cols] * self.dirs[cols].T[None, :, :]
        return out


def cubic_bspline(t: np.ndarray) -> np.ndarray:
    """Uniform cubic B-spline of unit knot spacing centred at 0 (support [-2, 2])."""
    a = np.abs(np.asarray(t, dtype=np.float64))
    return np.where(a < 1.0, (4.0 - 6.0 * a ** 2 + 3.0 * a ** 3) / 6.0,
                    np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def dipping_fault(mesh: Mesh, c: float, strike_range, dip_range, knots) -> Fault:
    """Unit-slip basis on the fault patch {y - z = c, x in strike_range,
    eta in dip_range} of a Kuhn lattice with equal spacing h on y and z:
    knots = (n_strike, n_dip) tensor-product cubic B-splines, each entirely
    inside the patch (so slip vanishes on its edges), each in the strike
    (1, 0, 0) and the up-dip (0, 1, 1)/sqrt 2 direction: 2 n_strike n_dip
    basis functions, strike ones first."""
    h = mesh.h
    if not np.isclose(h[1], h[2]):
        raise ValueError("the 45-degree fault needs equal y and z spacing")
    k = int(round(2.0 * c / h[1]))
    if k % 2 or not np.isclose(k * h[1] / 2.0, c):
        raise ValueError("c must be a whole number of lattice spacings")
    r = mesh.refined
    on = (r[:, 1] - r[:, 2]) == k
    x = mesh.xyz[:, 0]
    eta = (mesh.xyz[:, 1] + mesh.xyz[:, 2]) / np.sqrt(2.0)
    inside = on & (x >= strike_range[0] - 1e-12) & (x <= strike_range[1] + 1e-12) & \
        (eta >= dip_range[0] - 1e-12) & (eta <= dip_range[1] + 1e-12)
    nodes = np.nonzero(inside)[0]
    coords = np.stack([x[nodes], eta[nodes]], axis=1)
    touch = inside[mesh.conn].any(axis=1)
    d = (r[mesh.conn[:, :4], 1] - r[mesh.conn[:, :4], 2] - k).sum(axis=1)
    sides = np.where(touch, np.sign(d), 0).astype(np.int8)
    ns, nd = int(knots[0]), int(knots[1])
    hs = (strike_range[1] - strike_range[0]) / (ns + 3)
    hd = (dip_range[1] - dip_range[0]) / (nd + 3)
    cs = strike_range[0] + hs * (2 + np.arange(ns))
    cd = dip_range[0] + hd * (2 + np.arange(nd))
    bs = cubic_bspline((coords[:, 0:1] - cs[None, :]) / hs)  # (n_fault, ns)
    bd = cubic_bspline((coords[:, 1:2] - cd[None, :]) / hd)  # (n_fault, nd)
    one = (bs[:, :, None] * bd[:, None, :]).reshape(nodes.size, ns * nd)
    strike = np.array([1.0, 0.0, 0.0])
    dip = np.array([0.0, 1.0, 1.0]) / np.sqrt(2.0)
    normal = np.array([0.0, 1.0, -1.0]) / np.sqrt(2.0)
    basis = np.concatenate([one, one], axis=1)
    dirs = np.concatenate([np.tile(strike, (ns * nd, 1)), np.tile(dip, (ns * nd, 1))])
    return Fault(k=k, normal=normal, strike=strike, dip=dip, nodes=nodes, coords=coords, sides=sides,
                 basis=basis, dirs=dirs, knots=(ns, nd))


def laplacian_regularizer(ns: int, nd: int, ndir: int = 2) -> np.ndarray:
    """The regularisation operator of the inversion (an input of Eq. (5)):
    per slip direction, the five-point discrete Laplacian over the (ns x nd)
    grid of basis functions with zero slip beyond the grid; basis ordered
    direction-major, then (strike i, dip j) with j fastest, as in Fault."""
    n1 = ns * nd
    L = np.zeros((ndir * n1, ndir * n1))
    idx = np.arange(n1).reshape(ns, nd)
    for dct in range(ndir):
        o = dct * n1
        L[o + idx, o + idx] = 4.0
        L[o + idx[1:, :], o + idx[:-1, :]] = -1.0
        L[o + idx[:-1, :], o + idx[1:, :]] = -1.0
        L[o + idx[:, 1:], o + idx[:, :-1]] = -1.0
        L[o + idx[:, :-1], o + idx[:, 1:]] = -1.0
    return L


def surface_stations(mesh: Mesh, step: int) -> np.ndarray:
    """Top-surface nodes on every `step`-th corner line in x and y (refined
    coordinates multiples of 2 step, not on the domain's side faces): the
    observation points; each contributes its three displacement components."""
    r = mesh.refined
    top = r[:, 2] == 2 * mesh.grid[2]
    sel = top & (r[:, 0] % (2 * step) == 0) & (r[:, 1] % (2 * step) == 0) & \
        (r[:, 0] > 0) & (r[:, 1] > 0) & (r[:, 0] < 2 * mesh.grid[0]) & (r[:, 1] < 2 * mesh.grid[1])
    return np.nonzero(sel)[0]


def random_vectors(rng: np.random.Generator, n_nodes: int, nrhs: int, dtype=np.float64) -> np.ndarray:
    """(N, 3, nrhs) N(0, 1) input vectors (RHS index fastest)."""
    return rng.standard_normal((n_nodes, 3, nrhs)).astype(dtype)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
def cube_mesh(cfg_item_grid: int = 4) -> Mesh:
    """Small workload: unit cube, g^3 hexes, E=1, nu=0.25, bottom fixed."""
    g = cfg_item_grid
    m = kuhn_mesh(g, g, g)
    fix_faces(m, ((2, 0),))
    return m


def matvec_mesh(g: int = 64, seed_cfg: int = 2) -> Mesh:
    """EBE-matvec workload: unit cube, g^3 hexes, interior jitter 0.2h,
    three horizontal layers (E = 1, 3, 8; nu = 0.25, 0.27, 0.30), no BCs."""
    m = kuhn_mesh(g, g, g, jitter=0.2, rng=rng_for(seed_cfg, 0))
    set_layers_flat(m)
    return m


def crust_mesh(a: int = 96, b: int = 96, c: int = 48, seed_cfg: int = 3, jitter: float = 0.0) -> Mesh:
    """Multi-case crust workload: [0,2]x[0,2]x[0,1], three layers with seeded
    sinusoidal interfaces, bottom and four sides fixed, top free."""
    m = kuhn_mesh(a, b, c, lengths=(2.0, 2.0, 1.0), jitter=jitter,
                  rng=rng_for(seed_cfg, 9) if jitter > 0 else None)
    set_layers_sinusoidal(m, rng_for(seed_cfg, 1))
    fix_faces(m, BOX_SIDES_AND_BOTTOM)
    return m


def adjoint_mesh(a: int = 64, b: int = 64, c: int = 32, seed_cfg: int = 4) -> Mesh:
    """Adjoint workload: crust box, layered base times lognormal(0, 0.3)."""
    m = kuhn_mesh(a, b, c, lengths=(2.0, 2.0, 1.0))
    set_layers_sinusoidal(m, rng_for(seed_cfg, 1))
    lognormal_material(m, rng_for(seed_cfg, 2))
    fix_faces(m, BOX_SIDES_AND_BOTTOM)
    return m


def top_surface_dofs(mesh: Mesh) -> np.ndarray:
    """Flat DOF indices (node*3 + comp) of all top-surface DOFs."""
    top = face_nodes(mesh, 2, 1)
    return (3 * top[:, None] + np.arange(3)[None, :]).ravel()


def batch_sizes(rng: np.random.Generator, n_mesh: int = 32, lo: float = 5e4, hi: float = 2e6):
    """Log-uniform element targets -> (a, a, ceil(a/2)) grids and nrhs ~ U{1..16}."""
    T = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_mesh))
    a = np.maximum(2, np.round((T / 3.0) ** (1.0 / 3.0)).astype(int))
    grids = [(int(x), int(x), int(np.ceil(x / 2))) for x in a]
    nrhs = rng.integers(1, 17, size=n_mesh)
    return grids, [int(x) for x in nrhs]
