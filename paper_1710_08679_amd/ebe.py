"""Thin Python binding of the C ABI in ``include/ebe.h`` (``lib/libebe.so``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch CUDA tensors (PyTorch provides memory and
streams); vectors use the (nodes, 3, nrhs) layout, case index fastest.  The
library must be built (``python -m paper_1710_08679_amd.build``); nothing here
falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libebe.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_INDEX, ERR_INVERTED, ERR_CURVED, ERR_MATERIAL = -1, -2, -3, -4, -5
ERR_OOM, ERR_HIP, ERR_BREAKDOWN, ERR_NONFINITE, ERR_NUMBERING = -6, -7, -8, -9, -10
F64, F32 = 0, 1
PREC_PCGE, PREC_MG2, PREC_MG3 = 0, 1, 2
MODE_FP64, MODE_MIXED = 0, 1
MAX_RHS = 16
FORM_AUTO, FORM_GATHER, FORM_STAGED, FORM_PIPELINED, FORM_ASSEMBLED, FORM_COLOURED = -1, 0, 1, 2, 3, 4
FORM_DETERMINISTIC = 5
NUM_FORMS = 6

EXPORTED = (
    "ebe_mesh_create", "ebe_mesh_set_material", "ebe_mesh_info", "ebe_mesh_destroy", "ebe_matvec",
    "ebe_matvec_add",
    "ebe_matvec_p1", "ebe_prolong_p1", "ebe_restrict_p1", "ebe_diag_blocks", "ebe_block_jacobi",
    "ebe_pcg_default_opts", "ebe_pcg_solve", "ebe_adjoint_grad", "ebe_batch_create", "ebe_batch_solve",
    "ebe_batch_destroy", "ebe_status_string", "ebe_last_error", "ebe_build_info", "ebe_autotune",
    "ebe_set_product_form", "ebe_get_product_form", "ebe_level2_info", "ebe_matvec_l2", "ebe_prolong_l2",
    "ebe_restrict_l2", "ebe_matvec_noalloc", "ebe_patch_info", "ebe_set_product_variant",
    "ebe_get_product_variant", "ebe_fault_create", "ebe_fault_destroy", "ebe_split_node_forces",
    "ebe_greens_functions", "ebe_invert_lcurve", "ebe_batch_set_merge", "ebe_batch_info",
    "ebe_mesh_create_curved",
)


class PcgOpts(ctypes.Structure):
    _fields_ = [("precond", ctypes.c_int32), ("mode", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("inner_eps", ctypes.c_double * 3), ("inner_max", ctypes.c_int32 * 3),
                ("use_x0", ctypes.c_int32), ("coarse_guess", ctypes.c_int32), ("graphs", ctypes.c_int32),
                ("coarse_half", ctypes.c_int32), ("deterministic", ctypes.c_int32)]


class PcgStats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("inner_iters", ctypes.c_int64 * 3), ("max_rel_res", ctypes.c_double),
                ("seconds", ctypes.c_double), ("precond_used", ctypes.c_int32),
                ("graphs_captured", ctypes.c_int32), ("merged", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"outer_iters": self.outer_iters, "status": self.status,
                "inner_iters": [int(v) for v in self.inner_iters],
                "max_rel_res": self.max_rel_res, "seconds": self.seconds,
                "precond_used": self.precond_used, "graphs_captured": self.graphs_captured,
                "merged": self.merged}


class EbeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


_LIB = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


def load():
    """Load ``libebe.so``; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1710_08679_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "ebe_mesh_create": ([_vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)], _i32),
        "ebe_mesh_create_curved": ([_vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)], _i32),
        "ebe_mesh_set_material": ([_vp, _vp, _vp, _vp], _i32),
        "ebe_mesh_info": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)], _i32),
        "ebe_mesh_destroy": ([_vp], None),
        "ebe_patch_info": ([_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                            ctypes.POINTER(_i32)], _i32),
        "ebe_matvec": ([_vp, _i32, _i32, _vp, _vp, _i32, _vp], _i32),
        "ebe_matvec_add": ([_vp, _i32, _i32, _vp, _vp, _i32, _vp], _i32),
        "ebe_matvec_noalloc": ([_vp, _i32, _i32, _vp, _vp, _i32, _vp], _i32),
        "ebe_matvec_p1": ([_vp, _i32, _i32, _vp, _vp, _i32, _vp], _i32),
        "ebe_prolong_p1": ([_vp, _i32, _i32, _vp, _vp, _i32, _vp], _i32),
        "ebe_restrict_p1": ([_vp, _i32, _i32, _vp, _vp, _i32, _vp], _i32),
        "ebe_diag_blocks": ([_vp, _i32, _vp, _vp], _i32),
        "ebe_block_jacobi": ([_vp, _i32, _i32, _i32, _vp, _vp, _vp], _i32),
        "ebe_pcg_default_opts": ([ctypes.POINTER(PcgOpts)], None),
        "ebe_pcg_solve": ([_vp, _i32, _vp, _vp, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgStats), _vp], _i32),
        "ebe_adjoint_grad": ([_vp, _i32, _i32, _vp, _vp, _vp, _vp], _i32),
        "ebe_batch_create": ([ctypes.POINTER(_vp), _i32, ctypes.POINTER(_i32), ctypes.POINTER(_vp)], _i32),
        "ebe_batch_solve": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(PcgOpts),
                             ctypes.POINTER(PcgStats), _vp], _i32),
        "ebe_batch_destroy": ([_vp], None),
        "ebe_batch_set_merge": ([_vp, _i64], _i32),
        "ebe_batch_info": ([_vp, ctypes.POINTER(_i32), _vp], _i32),
        "ebe_status_string": ([_i32], ctypes.c_char_p),
        "ebe_last_error": ([], ctypes.c_char_p),
        "ebe_build_info": ([], ctypes.c_char_p),
        "ebe_autotune": ([_vp, _i32, _i32, _i32, _vp, ctypes.POINTER(ctypes.c_double)], _i32),
        "ebe_set_product_form": ([_vp, _i32, _i32, _i32, _i32], _i32),
        "ebe_get_product_form": ([_vp, _i32, _i32, _i32, ctypes.POINTER(_i32)], _i32),
        "ebe_set_product_variant": ([_vp, _i32, _i32, _i32, _i32], _i32),
        "ebe_fault_create": ([_vp, _vp, _i64, _vp, _i32, _vp, _vp, ctypes.POINTER(_vp)], _i32),
        "ebe_fault_destroy": ([_vp], None),
        "ebe_split_node_forces": ([_vp, _i32, _i32, _vp, _vp], _i32),
        "ebe_greens_functions": ([_vp, _i32, _vp, _vp, ctypes.POINTER(PcgOpts), _vp, _vp], _i32),
        "ebe_invert_lcurve": ([_i32, _i32, _vp, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
        "ebe_get_product_variant": ([_vp, _i32, _i32, _i32, ctypes.POINTER(_i32)], _i32),
        "ebe_level2_info": ([_vp, ctypes.POINTER(_i64), _vp], _i32),
        "ebe_matvec_l2": ([_vp, _i32, _i32, _vp, _vp, _i32, _vp], _i32),
        "ebe_prolong_l2": ([_vp, _i32, _i32, _vp, _vp, _vp], _i32),
        "ebe_restrict_l2": ([_vp, _i32, _i32, _vp, _vp, _vp], _i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = lib
    return lib


def _check(status: int) -> int:
    if status < 0:
        lib = load()
        raise EbeError(status, f"{lib.ebe_status_string(status).decode()}: {lib.ebe_last_error().decode()}")
    return status


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _dtype_code(dtype) -> int:
    """F64 / F32 from an ebe code or a torch dtype."""
    import torch
    if dtype in (F64, F32):
        return int(dtype)
    if dtype == torch.float64:
        return F64
    if dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {dtype!r}")


def _dev(t, dtype=None, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return _vp(t.data_ptr())


def _dtype_code(dtype) -> int:
    import torch
    if dtype == torch.float64:
        return F64
    if dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {dtype}: float64 or float32")


def default_opts(**kw) -> PcgOpts:
    o = PcgOpts()
    load().ebe_pcg_default_opts(ctypes.byref(o))
    names = {f[0] for f in PcgOpts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown solver option {k!r}")
        if k in ("inner_eps", "inner_max"):
            for i, x in enumerate(v):  # levels 0, 1 (and 2)
                getattr(o, k)[i] = x
        else:
            setattr(o, k, v)
    return o


class Mesh:
    """A device-resident mesh handle (``ebe_mesh``)."""

    def __init__(self, xyz, conn, n_vertices, young, poisson, fixed=None, stream=None, curved=False):
        """curved: create with ``ebe_mesh_create_curved`` (isoparametric elements,
        edge nodes anywhere) instead of ``ebe_mesh_create`` (straight-sided)."""
        lib = load()
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        young = np.ascontiguousarray(young, dtype=np.float64)
        poisson = np.ascontiguousarray(poisson, dtype=np.float64)
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        self.n_nodes, self.n_vertices, self.n_elem = int(xyz.shape[0]), int(n_vertices), int(conn.shape[0])
        if xyz.shape != (self.n_nodes, 3) or conn.shape != (self.n_elem, 10):
            raise ValueError("xyz must be (N, 3) and conn (E, 10)")
        if young.shape != (self.n_elem,) or poisson.shape != (self.n_elem,):
            raise ValueError("young and poisson must be (E,)")
        if fx is not None and fx.shape != (self.n_nodes, 3):
            raise ValueError("fixed must be (N, 3)")
        h = _vp()
        create = lib.ebe_mesh_create_curved if curved else lib.ebe_mesh_create
        _check(create(xyz.ctypes.data, self.n_nodes, self.n_vertices, conn.ctypes.data, self.n_elem,
                      young.ctypes.data, poisson.ctypes.data, None if fx is None else fx.ctypes.data,
                      _vp(None) if stream is None else _stream(stream), ctypes.byref(h)))
        self.curved = bool(curved)
        self._h = h

    @classmethod
    def from_generated(cls, m, stream=None, curved=False) -> "Mesh":
        """Upload a ``meshgen.Mesh`` (curved: as isoparametric elements)."""
        fixed = m.fixed if m.fixed.any() else None
        return cls(m.xyz, m.conn, m.n_vertices, m.young, m.poisson, fixed, stream, curved=curved)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("mesh handle was destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().ebe_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n, nv, ne = _i64(), _i64(), _i64()
        _check(load().ebe_mesh_info(self.handle, ctypes.byref(n), ctypes.byref(nv), ctypes.byref(ne)))
        return n.value, nv.value, ne.value

    def patch_info(self, level=0):
        """dict: patches, shared nodes, staged partial-sum rows and colours of a level's products."""
        npat, nsh, nst, ncol = _i64(), _i64(), _i64(), _i32()
        _check(load().ebe_patch_info(self.handle, int(level), ctypes.byref(npat), ctypes.byref(nsh),
                                     ctypes.byref(nst), ctypes.byref(ncol)))
        return {"patches": npat.value, "shared": nsh.value, "staged": nst.value, "colours": ncol.value}

    # ---- operators -------------------------------------------------------
    def _vec_op(self, fn, x, rows_in, rows_out, apply_bc, out, stream):
        import torch
        if x.dim() != 3 or x.shape[0] != rows_in or x.shape[1] != 3:
            raise ValueError(f"x must be ({rows_in}, 3, nrhs)")
        nrhs = int(x.shape[2])
        if out is None:
            out = torch.empty((rows_out, 3, nrhs), dtype=x.dtype, device=x.device)
        _check(fn(self.handle, _dtype_code(x.dtype), nrhs, _dev(x, name="x"),
                  _dev(out, x.dtype, (rows_out, 3, nrhs), "out"), int(bool(apply_bc)), _stream(stream)))
        return out

    def autotune(self, level, dtype, nrhs, stream=None):
        """Time every product form for (level, dtype, nrhs) and keep the fastest;
        returns the times in ms, indexed by form (-1: no such form at this level;
        FORM_ASSEMBLED exists at the linear level only, FORM_COLOURED at the quadratic level only)."""
        ms = (ctypes.c_double * NUM_FORMS)()
        _check(load().ebe_autotune(self.handle, int(level), _dtype_code(dtype), int(nrhs), _stream(stream), ms))
        return tuple(float(v) for v in ms)

    def set_form(self, level, dtype, nrhs, form):
        _check(load().ebe_set_product_form(self.handle, int(level), _dtype_code(dtype), int(nrhs), int(form)))

    def set_variant(self, level, dtype, nrhs, variant):
        _check(load().ebe_set_product_variant(self.handle, int(level), _dtype_code(dtype), int(nrhs), int(variant)))

    def variant(self, level, dtype, nrhs):
        v = _i32()
        _check(load().ebe_get_product_variant(self.handle, int(level), _dtype_code(dtype), int(nrhs),
                                              ctypes.byref(v)))
        return int(v.value)

    def form(self, level, dtype, nrhs):
        f = _i32()
        _check(load().ebe_get_product_form(self.handle, int(level), _dtype_code(dtype), int(nrhs), ctypes.byref(f)))
        return int(f.value)

    def matvec(self, x, apply_bc=False, out=None, stream=None):
        """y = K x (quadratic elements); x (N, 3, nrhs) float64/float32."""
        return self._vec_op(load().ebe_matvec, x, self.n_nodes, self.n_nodes, apply_bc, out, stream)

    def matvec_noalloc(self, x, apply_bc=False, out=None, stream=None):
        """y = K x through the allocation-free entry point (out may be preallocated)."""
        return self._vec_op(load().ebe_matvec_noalloc, x, self.n_nodes, self.n_nodes, apply_bc, out, stream)

    def matvec_add(self, x, y, apply_bc=False, stream=None):
        """y += K x (in place); returns y."""
        return self._vec_op(load().ebe_matvec_add, x, self.n_nodes, self.n_nodes, apply_bc, y, stream)

    def matvec_p1(self, x, apply_bc=False, out=None, stream=None):
        """y = K1 x on the corner-only linear mesh; x (Nv, 3, nrhs)."""
        return self._vec_op(load().ebe_matvec_p1, x, self.n_vertices, self.n_vertices, apply_bc, out, stream)

    def prolong(self, x, apply_bc=False, out=None, stream=None):
        """y (N, 3, n) = P1 x (Nv, 3, n)."""
        return self._vec_op(load().ebe_prolong_p1, x, self.n_vertices, self.n_nodes, apply_bc, out, stream)

    def restrict(self, x, apply_bc=False, out=None, stream=None):
        """y (Nv, 3, n) = P1^T x (N, 3, n)."""
        return self._vec_op(load().ebe_restrict_p1, x, self.n_nodes, self.n_vertices, apply_bc, out, stream)

    # ---- level 2 (aggregates of the corner mesh) --------------------------
    def level2_info(self):
        """(n_agg, agg) with agg (Nv,) int32: each corner's aggregate."""
        na = _i64()
        agg = np.empty(self.n_vertices, dtype=np.int32)
        _check(load().ebe_level2_info(self.handle, ctypes.byref(na), agg.ctypes.data))
        return int(na.value), agg

    @property
    def n_agg(self):
        na = _i64()
        _check(load().ebe_level2_info(self.handle, ctypes.byref(na), None))
        return int(na.value)

    def matvec_l2(self, x, apply_bc=False, out=None, stream=None):
        """y = A2 x on the aggregates; x (Na, 3, nrhs)."""
        na = self.n_agg
        return self._vec_op(load().ebe_matvec_l2, x, na, na, apply_bc, out, stream)

    def prolong_l2(self, x, out=None, stream=None):
        """y (Nv, 3, n) = P2 x (Na, 3, n)."""
        return self._vec_op2(load().ebe_prolong_l2, x, self.n_agg, self.n_vertices, out, stream)

    def restrict_l2(self, x, out=None, stream=None):
        """y (Na, 3, n) = P2^T x (Nv, 3, n)."""
        return self._vec_op2(load().ebe_restrict_l2, x, self.n_vertices, self.n_agg, out, stream)

    def _vec_op2(self, fn, x, rows_in, rows_out, out, stream):
        import torch
        if x.dim() != 3 or x.shape[0] != rows_in or x.shape[1] != 3:
            raise ValueError(f"x must be ({rows_in}, 3, nrhs)")
        nrhs = int(x.shape[2])
        if out is None:
            out = torch.empty((rows_out, 3, nrhs), dtype=x.dtype, device=x.device)
        _check(fn(self.handle, _dtype_code(x.dtype), nrhs, _dev(x, name="x"),
                  _dev(out, x.dtype, (rows_out, 3, nrhs), "out"), _stream(stream)))
        return out

    def _rows(self, level):
        return (self.n_nodes, self.n_vertices, self.n_agg)[level]

    def block_jacobi(self, x, level=0, out=None, stream=None):
        import torch
        rows = self._rows(level)
        if x.dim() != 3 or x.shape[0] != rows or x.shape[1] != 3:
            raise ValueError(f"x must be ({rows}, 3, nrhs)")
        nrhs = int(x.shape[2])
        if out is None:
            out = torch.empty_like(x)
        _check(load().ebe_block_jacobi(self.handle, int(level), _dtype_code(x.dtype), nrhs, _dev(x, name="x"),
                                       _dev(out, x.dtype, x.shape, "out"), _stream(stream)))
        return out

    def diag_blocks(self, level=0, stream=None):
        """(rows, 3, 3) float64 nodal diagonal blocks (level 0, 1 or 2)."""
        import torch
        rows = self._rows(level)
        out = torch.empty((rows, 3, 3), dtype=torch.float64, device="cuda")
        _check(load().ebe_diag_blocks(self.handle, int(level), _dev(out), _stream(stream)))
        return out

    def set_material(self, young, poisson, stream=None):
        import torch
        _check(load().ebe_mesh_set_material(self.handle, _dev(young, torch.float64, (self.n_elem,), "young"),
                                            _dev(poisson, torch.float64, (self.n_elem,), "poisson"),
                                            _stream(stream)))

    def adjoint_grad(self, u, lam, out=None, stream=None):
        """g_e = -sum_c lam_{c,e}^T (K_e/E_e) u_{c,e}; u, lam (N, 3, nrhs) of one dtype."""
        import torch
        if u.shape != lam.shape or u.dtype != lam.dtype or u.dim() != 3 or u.shape[0] != self.n_nodes:
            raise ValueError("u and lam must both be (N, 3, nrhs) of one dtype")
        nrhs = int(u.shape[2])
        if out is None:
            out = torch.empty((self.n_elem,), dtype=u.dtype, device=u.device)
        _check(load().ebe_adjoint_grad(self.handle, _dtype_code(u.dtype), nrhs, _dev(u, name="u"),
                                       _dev(lam, name="lam"), _dev(out, u.dtype, (self.n_elem,), "out"),
                                       _stream(stream)))
        return out

    def solve(self, f, u=None, opts: PcgOpts | None = None, stream=None, raise_on_nonconv=False, **kw):
        """Solve P K P u = P f for f (N, 3, nrhs) float64; returns (u, stats dict)."""
        import torch
        if f.dim() != 3 or f.shape[0] != self.n_nodes or f.shape[1] != 3:
            raise ValueError("f must be (N, 3, nrhs)")
        nrhs = int(f.shape[2])
        if u is None:
            u = torch.empty_like(f)
        if opts is None:
            opts = default_opts(**kw)
        st = PcgStats()
        status = _check(load().ebe_pcg_solve(self.handle, nrhs, _dev(f, torch.float64, name="f"),
                                             _dev(u, torch.float64, f.shape, "u"), ctypes.byref(opts),
                                             ctypes.byref(st), _stream(stream)))
        if raise_on_nonconv and status == NOT_CONVERGED:
            raise EbeError(status, f"not converged: {st.as_dict()}")
        return u, st.as_dict()


def batch_solve(meshes, fs, us=None, opts: PcgOpts | None = None, stream=None, merge_elems=None, info=None,
                **kw):
    """Solve several meshes (each with its own nrhs) as one batch; returns (us, [stats]).
    merge_elems: merge meshes up to this many elements (None: the library default, 0: none);
    info: a dict that receives the merged groups ({"groups": g, "group_of": [...]})."""
    import torch
    lib = load()
    n = len(meshes)
    if us is None:
        us = [torch.empty_like(f) for f in fs]
    for m, f, u in zip(meshes, fs, us):
        if f.shape != (m.n_nodes, 3, f.shape[2]) or u.shape != f.shape:
            raise ValueError("each f / u must be (N_i, 3, nrhs_i)")
        _dev(f, torch.float64, name="f")
        _dev(u, torch.float64, name="u")
    hs = (_vp * n)(*[m.handle for m in meshes])
    nr = (_i32 * n)(*[int(f.shape[2]) for f in fs])
    b = _vp()
    _check(lib.ebe_batch_create(hs, n, nr, ctypes.byref(b)))
    try:
        if merge_elems is not None:
            _check(lib.ebe_batch_set_merge(b, int(merge_elems)))
        if info is not None:
            ng = _i32()
            gof = np.empty(n, dtype=np.int32)
            _check(lib.ebe_batch_info(b, ctypes.byref(ng), gof.ctypes.data))
            info["groups"], info["group_of"] = int(ng.value), gof.tolist()
        fp = (_vp * n)(*[f.data_ptr() for f in fs])
        up = (_vp * n)(*[u.data_ptr() for u in us])
        st = (PcgStats * n)()
        if opts is None:
            opts = default_opts(**kw)
        _check(lib.ebe_batch_solve(b, fp, up, ctypes.byref(opts), st, _stream(stream)))
    finally:
        lib.ebe_batch_destroy(b)
    return us, [s.as_dict() for s in st]


class Fault:
    """A fault with unit-slip basis functions on a mesh (``ebe_fault``):
    split-node forces and Green's functions at observation points."""

    def __init__(self, mesh: "Mesh", sides, nodes, basis, dirs):
        lib = load()
        sides = np.ascontiguousarray(sides, dtype=np.int8)
        nodes = np.ascontiguousarray(nodes, dtype=np.int32)
        basis = np.ascontiguousarray(basis, dtype=np.float64)
        dirs = np.ascontiguousarray(dirs, dtype=np.float64)
        if sides.shape != (mesh.n_elem,) or basis.shape[0] != nodes.size or dirs.shape != (basis.shape[1], 3):
            raise ValueError("sides (E,), basis (n_fault_nodes, n_basis), dirs (n_basis, 3)")
        self.mesh, self.n_basis = mesh, int(basis.shape[1])
        h = _vp()
        _check(lib.ebe_fault_create(mesh.handle, sides.ctypes.data, nodes.size, nodes.ctypes.data, self.n_basis,
                                    basis.ctypes.data, dirs.ctypes.data, ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_generated(cls, mesh: "Mesh", flt) -> "Fault":
        """From a ``meshgen.Fault``."""
        return cls(mesh, flt.sides, flt.nodes, flt.basis, flt.dirs)

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().ebe_fault_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def split_node_forces(self, col0, nrhs, out=None, stream=None):
        """f (N, 3, nrhs) float64: split-node forces of basis functions col0 .. col0 + nrhs - 1."""
        import torch
        if out is None:
            out = torch.empty((self.mesh.n_nodes, 3, nrhs), dtype=torch.float64, device="cuda")
        _check(load().ebe_split_node_forces(self._h, int(col0), int(nrhs),
                                            _dev(out, torch.float64, (self.mesh.n_nodes, 3, nrhs), "out"),
                                            _stream(stream)))
        return out

    def greens_functions(self, stations, opts: PcgOpts | None = None, stream=None, **kw):
        """(G (3 m, n_basis) float64 on the device, [per-set stats]) for the m station nodes."""
        import torch
        st = np.ascontiguousarray(stations, dtype=np.int32)
        G = torch.empty((3 * st.size, self.n_basis), dtype=torch.float64, device="cuda")
        nset = (self.n_basis + MAX_RHS - 1) // MAX_RHS
        stats = (PcgStats * nset)()
        if opts is None:
            opts = default_opts(**kw)
        _check(load().ebe_greens_functions(self._h, st.size, st.ctypes.data, _dev(G), ctypes.byref(opts), stats,
                                           _stream(stream)))
        return G, [x.as_dict() for x in stats]


def invert_lcurve(G, d, L, alphas, stream=None):
    """Eq. (5) over the weights: returns (a (n_alpha, n_basis), rho, eta, curvature, corner) on the device
    (curvature and corner None with fewer than three weights).  G (n_obs, n_basis), d (n_obs,),
    L (n_reg, n_basis): float64 CUDA tensors; alphas: host sequence, positive and increasing."""
    import torch
    al = np.ascontiguousarray(alphas, dtype=np.float64)
    nobs, nb = G.shape
    nreg = L.shape[0]
    _dev(G, torch.float64, (nobs, nb), "G")
    _dev(d, torch.float64, (nobs,), "d")
    _dev(L, torch.float64, (nreg, nb), "L")
    a = torch.empty((al.size, nb), dtype=torch.float64, device=G.device)
    rho = torch.empty(al.size, dtype=torch.float64, device=G.device)
    eta = torch.empty_like(rho)
    curv = torch.empty_like(rho) if al.size >= 3 else None
    corner = torch.empty(1, dtype=torch.int32, device=G.device) if al.size >= 3 else None
    _check(load().ebe_invert_lcurve(nobs, nb, _dev(G), _dev(d), nreg, _dev(L), al.size, al.ctypes.data, _dev(a),
                                    _dev(rho), _dev(eta), None if curv is None else _dev(curv),
                                    None if corner is None else _dev(corner), _stream(stream)))
    return a, rho, eta, curv, (None if corner is None else int(corner.item()))
