"""skelfmm on MI355X: fast summation u = A q, A_ij = G(x_i, x_j), by the
neighbor-list skeletonization FMM (arXiv 2310.16668).

Thin Python binding over the C ABI in ``include/skelfmm.h``: argument
marshalling only.  The build runs in the library's host code; every step of an
apply runs in the library's HIP kernels on the caller's current stream.  If the
compiled library is missing, importing this package fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SKELFMM_LIB selects another build of the same library (the host-sanitizer build)
_LIB_PATH = os.environ.get("SKELFMM_LIB") or os.path.join(_HERE, "libskelfmm.so")

if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing; build it with __graft_entry__.build() "
                      "or python paper_2310_16668_amd/_build.py")

# torch ships its own HIP runtime under the same soname as the system one; load
# torch first so this library binds to the runtime that owns torch's device
# memory and streams (one HIP runtime per process).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(_LIB_PATH)

LAPLACE, HELMHOLTZ = 0, 1
F64, F32, C128, C64 = 0, 1, 2, 3
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOTSUP", -5: "EINTERNAL"}


class SkelfmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dim", ctypes.c_int32), ("kappa", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("proxy_shape", ctypes.c_int32), ("proxy_points", ctypes.c_int32),
                ("proxy_scale", ctypes.c_double), ("no_compression", ctypes.c_int32),
                ("num_threads", ctypes.c_int32), ("keep_transparent", ctypes.c_int32),
                ("f64_leaf", ctypes.c_int32), ("nonsymmetric", ctypes.c_int32), ("no_expansion", ctypes.c_int32),
                ("compensated_leaf", ctypes.c_int32), ("gpu_build", ctypes.c_int32),
                ("f32_differences", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class Stats(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_boxes", ctypes.c_int32), ("n_leaves", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("top_level", ctypes.c_int32), ("k_max", ctypes.c_int32),
                ("proxy_count", ctypes.c_int32), ("t_tree", ctypes.c_double), ("t_skel", ctypes.c_double),
                ("m_proj_elems", ctypes.c_int64), ("n_entries", ctypes.c_int64),
                ("pairs_near", ctypes.c_int64), ("pairs_skel", ctypes.c_int64), ("n_tasks", ctypes.c_int64),
                ("tile_targets", ctypes.c_int32), ("n_sym_tasks", ctypes.c_int32), ("pairs_sym", ctypes.c_int64),
                ("pairs_sym_skel", ctypes.c_int64), ("pairs_tile", ctypes.c_int64),
                ("pairs_tile_skel", ctypes.c_int64), ("n_sym_expanded", ctypes.c_int32),
                ("n_sym_f32diff", ctypes.c_int32), ("t_skel_qr", ctypes.c_double), ("t_layout", ctypes.c_double)]


_P = ctypes.POINTER


class PlanView(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("kind", ctypes.c_int32), ("kappa", ctypes.c_double),
                ("n_points", ctypes.c_int64), ("points", _P(ctypes.c_double)),
                ("n_boxes", ctypes.c_int32), ("max_level", ctypes.c_int32), ("top_level", ctypes.c_int32),
                ("pad0", ctypes.c_int32),
                ("level", _P(ctypes.c_int32)), ("parent", _P(ctypes.c_int32)), ("is_leaf", _P(ctypes.c_int32)),
                ("child_ptr", _P(ctypes.c_int32)), ("child_idx", _P(ctypes.c_int32)), ("coord", _P(ctypes.c_int32)),
                ("idx_ptr", _P(ctypes.c_int64)), ("idx", _P(ctypes.c_int64)), ("pos", _P(ctypes.c_int64)),
                ("rank", _P(ctypes.c_int32)), ("T_ptr", _P(ctypes.c_int64)), ("T", _P(ctypes.c_double)),
                ("coll_ptr", _P(ctypes.c_int32)), ("coll_idx", _P(ctypes.c_int32)),
                ("coarse_ptr", _P(ctypes.c_int32)), ("coarse_idx", _P(ctypes.c_int32)),
                ("fine_ptr", _P(ctypes.c_int32)), ("fine_idx", _P(ctypes.c_int32)),
                ("root_lo", ctypes.c_double * 3), ("root_side", ctypes.c_double)]


_vp = ctypes.c_void_p
_lib.skelfmm_build.argtypes = [_P(ctypes.c_double), ctypes.c_int64, Kernel, ctypes.c_double, ctypes.c_int32,
                               _P(Options), _P(_vp)]
_lib.skelfmm_prepare.argtypes = [_vp, ctypes.c_int64, ctypes.c_int]
_lib.skelfmm_apply.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int, _vp]
_lib.skelfmm_apply_adjoint.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int, _vp]
_lib.skelfmm_stats_get.argtypes = [_vp, _P(Stats)]
_lib.skelfmm_export.argtypes = [_vp, _P(PlanView)]
_lib.skelfmm_batch_create.argtypes = [_P(_vp), ctypes.c_int32, _P(_vp)]
_lib.skelfmm_batch_apply.argtypes = [_vp, _P(_vp), _P(_vp), ctypes.c_int64, ctypes.c_int, ctypes.c_int32, _vp]
_lib.skelfmm_batch_destroy.argtypes = [_vp]
_lib.skelfmm_destroy.argtypes = [_vp]
_lib.skelfmm_timing.argtypes = [_vp, ctypes.c_int32]
_lib.skelfmm_autotune.argtypes = [_vp, ctypes.c_int, _vp, _P(ctypes.c_int32), _P(ctypes.c_float)]
_lib.skelfmm_set_targets_per_lane.argtypes = [_vp, ctypes.c_int32]
_lib.skelfmm_autotune_transfers.argtypes = [_vp, ctypes.c_int64, _vp, _P(ctypes.c_int32), _P(ctypes.c_float)]
_lib.skelfmm_set_transfer_shape.argtypes = [_vp, ctypes.c_int32]
_lib.skelfmm_batch_autotune_transfers.argtypes = [_vp, ctypes.c_int64, _vp, _P(ctypes.c_int32), _P(ctypes.c_float)]
_lib.skelfmm_timing_read.argtypes = [_vp, _P(ctypes.c_double), _P(ctypes.c_int64)]
_lib.skelfmm_batch_timing.argtypes = [_vp, ctypes.c_int32]
_lib.skelfmm_batch_timing.restype = ctypes.c_int
_lib.skelfmm_batch_timing_read.argtypes = [_vp, _P(ctypes.c_double), _P(ctypes.c_int64)]
_lib.skelfmm_batch_timing_read.restype = ctypes.c_int
_lib.skelfmm_apply_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int32, _vp]
_lib.skelfmm_apply_noalloc.restype = ctypes.c_int
_lib.skelfmm_apply_fwd_adj.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp]
_lib.skelfmm_apply_fwd_adj.restype = ctypes.c_int
_lib.skelfmm_autotune_fwd_adj.argtypes = [_vp, _vp, _P(ctypes.c_int32), _P(ctypes.c_float)]
_lib.skelfmm_autotune_fwd_adj.restype = ctypes.c_int
_lib.skelfmm_noalloc_scratch_bytes.argtypes = []
_lib.skelfmm_noalloc_scratch_bytes.restype = ctypes.c_int64
_lib.skelfmm_last_error.restype = ctypes.c_char_p
for _f in ("skelfmm_build", "skelfmm_prepare", "skelfmm_apply", "skelfmm_apply_adjoint", "skelfmm_stats_get",
           "skelfmm_export", "skelfmm_batch_create", "skelfmm_batch_apply", "skelfmm_timing",
           "skelfmm_timing_read", "skelfmm_autotune", "skelfmm_set_targets_per_lane", "skelfmm_autotune_transfers",
           "skelfmm_set_transfer_shape", "skelfmm_batch_autotune_transfers"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ("skelfmm_build", "skelfmm_prepare", "skelfmm_apply", "skelfmm_apply_adjoint", "skelfmm_stats_get",
            "skelfmm_export", "skelfmm_batch_create", "skelfmm_batch_apply", "skelfmm_batch_destroy",
            "skelfmm_destroy", "skelfmm_last_error", "skelfmm_timing", "skelfmm_timing_read",
            "skelfmm_autotune", "skelfmm_set_targets_per_lane", "skelfmm_autotune_transfers",
            "skelfmm_set_transfer_shape", "skelfmm_batch_autotune_transfers", "skelfmm_batch_timing",
            "skelfmm_batch_timing_read", "skelfmm_apply_noalloc",
            "skelfmm_noalloc_scratch_bytes", "skelfmm_apply_fwd_adj", "skelfmm_autotune_fwd_adj")
NXFER = 4
PASSES = ("gather", "upward", "near_field", "near_pairs", "near_reduce", "downward", "output")


def _check(status: int):
    if status != 0:
        raise SkelfmmError(status, _lib.skelfmm_last_error().decode())


def library_path() -> str:
    return _LIB_PATH


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    m = {torch.float64: F64, torch.float32: F32, torch.complex128: C128, torch.complex64: C64}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


class Operator:
    """A built skeleton operator: ``apply(q) = Atilde q``, ``apply_adjoint(v) = Atilde^H v``."""

    def __init__(self, handle, n: int, dim: int, kind: int):
        self._h = handle
        self._destroy = _lib.skelfmm_destroy   # kept: module globals may be gone at exit
        self.n, self.dim, self.kind = n, dim, kind

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        s = Stats()
        _check(_lib.skelfmm_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_ if f != "reserved"}

    def export(self) -> dict:
        """Copies of the skeleton operators as numpy arrays (read through skelfmm_export)."""
        v = PlanView()
        _check(_lib.skelfmm_export(self._h, ctypes.byref(v)))
        nb, n = v.n_boxes, v.n_points

        def arr(ptr, count, dt):
            if count == 0:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dt, copy=True)

        child_ptr = arr(v.child_ptr, nb + 1, np.int32)
        idx_ptr = arr(v.idx_ptr, nb + 1, np.int64)
        T_ptr = arr(v.T_ptr, nb + 1, np.int64)
        coll_ptr = arr(v.coll_ptr, nb + 1, np.int32)
        coarse_ptr = arr(v.coarse_ptr, nb + 1, np.int32)
        fine_ptr = arr(v.fine_ptr, nb + 1, np.int32)
        return {
            "dim": v.dim, "kind": "helmholtz" if v.kind == HELMHOLTZ else "laplace", "kappa": v.kappa,
            "points": arr(v.points, n * v.dim, np.float64).reshape(n, v.dim),
            "n_boxes": nb, "max_level": v.max_level, "top_level": v.top_level,
            "level": arr(v.level, nb, np.int32), "parent": arr(v.parent, nb, np.int32),
            "is_leaf": arr(v.is_leaf, nb, np.int32), "child_ptr": child_ptr,
            "child_idx": arr(v.child_idx, int(child_ptr[-1]), np.int32),
            "coord": arr(v.coord, 3 * nb, np.int32).reshape(nb, 3),
            "idx_ptr": idx_ptr, "idx": arr(v.idx, int(idx_ptr[-1]), np.int64),
            "pos": arr(v.pos, int(idx_ptr[-1]), np.int64), "rank": arr(v.rank, nb, np.int32),
            "T_ptr": T_ptr, "T": arr(v.T, int(T_ptr[-1]), np.float64),
            "coll_ptr": coll_ptr, "coll_idx": arr(v.coll_idx, int(coll_ptr[-1]), np.int32),
            "coarse_ptr": coarse_ptr, "coarse_idx": arr(v.coarse_idx, int(coarse_ptr[-1]), np.int32),
            "fine_ptr": fine_ptr, "fine_idx": arr(v.fine_idx, int(fine_ptr[-1]), np.int32),
            "root_lo": np.array(v.root_lo[:]), "root_side": v.root_side,
        }

    def autotune(self, dtype=None) -> dict:
        """Time the near-field launches with 1 .. 4 targets per lane; keep the fastest."""
        torch = _torch()
        if dtype is None:
            dtype = torch.complex128 if self.kind == HELMHOLTZ else torch.float64
        code = _dtype_code(torch.empty(0, dtype=dtype))
        chosen = ctypes.c_int32()
        ms = (ctypes.c_float * 4)()
        stream = torch.cuda.current_stream().cuda_stream
        _check(_lib.skelfmm_autotune(self._h, code, stream, ctypes.byref(chosen), ms))
        return {"targets_per_lane": chosen.value, "ms": {t: ms[t - 1] for t in (1, 2, 3, 4)}}

    def set_targets_per_lane(self, tpl: int):
        _check(_lib.skelfmm_set_targets_per_lane(self._h, tpl))

    def autotune_transfers(self, nrhs: int) -> dict:
        """Time the float32 many-RHS matrix-core transfers in every launch shape; keep the fastest."""
        torch = _torch()
        chosen = ctypes.c_int32()
        ms = (ctypes.c_float * NXFER)()
        _check(_lib.skelfmm_autotune_transfers(self._h, nrhs, torch.cuda.current_stream().cuda_stream,
                                               ctypes.byref(chosen), ms))
        return {"shape": chosen.value, "ms": [ms[i] for i in range(NXFER)]}

    def set_transfer_shape(self, shape: int):
        _check(_lib.skelfmm_set_transfer_shape(self._h, shape))

    def timing(self, enable: bool = True):
        """Enable (and zero) or disable per-pass HIP-event timing of applies."""
        _check(_lib.skelfmm_timing(self._h, int(enable)))

    def timing_read(self) -> dict:
        """Summed milliseconds per pass over the timed applies (waits for them)."""
        ms = (ctypes.c_double * len(PASSES))()
        n = ctypes.c_int64()
        _check(_lib.skelfmm_timing_read(self._h, ms, ctypes.byref(n)))
        out = {p: ms[i] for i, p in enumerate(PASSES)}
        out["sweeps"] = n.value
        return out

    def prepare(self, nrhs: int = 1, dtype=None):
        torch = _torch()
        if dtype is None:
            dtype = torch.complex128 if self.kind == HELMHOLTZ else torch.float64
        code = _dtype_code(torch.empty(0, dtype=dtype))
        _check(_lib.skelfmm_prepare(self._h, nrhs, code))

    def _run(self, q, adjoint: bool):
        torch = _torch()
        if not q.is_cuda:
            raise ValueError("apply takes a device tensor")
        squeeze = q.dim() == 1
        q2 = q.reshape(q.shape[0], -1).contiguous()
        if q2.shape[0] != self.n:
            raise ValueError(f"expected {self.n} rows, got {q2.shape[0]}")
        u = torch.empty_like(q2)
        stream = torch.cuda.current_stream(q2.device).cuda_stream
        fn = _lib.skelfmm_apply_adjoint if adjoint else _lib.skelfmm_apply
        _check(fn(self._h, q2.data_ptr(), u.data_ptr(), q2.shape[1], _dtype_code(q2), stream))
        return u[:, 0] if squeeze else u

    def apply(self, q):
        """u = Atilde q for a device tensor q of shape [n] or [n, nrhs]."""
        return self._run(q, False)

    def apply_noalloc(self, q, out, adjoint: bool = False):
        """Atilde q (or Atilde^H q) into the caller's tensor ``out`` with the library's
        static scratch workspace (skelfmm_apply_noalloc): no device allocation.  The
        operator must be uploaded for q's dtype first (``prepare(0, dtype)``)."""
        torch = _torch()
        if not (q.is_cuda and out.is_cuda) or not (q.is_contiguous() and out.is_contiguous()):
            raise ValueError("q and out must be contiguous device tensors")
        if q.shape != out.shape or q.dtype != out.dtype or q.shape[0] != self.n:
            raise ValueError("q and out must have the same shape and dtype, with n rows")
        nrhs = 1 if q.dim() == 1 else q.shape[1]
        stream = torch.cuda.current_stream(q.device).cuda_stream
        _check(_lib.skelfmm_apply_noalloc(self._h, q.data_ptr(), out.data_ptr(), nrhs, _dtype_code(q),
                                          int(adjoint), stream))
        return out

    def apply_adjoint(self, v):
        """w = Atilde^H v (the transposed sweep)."""
        return self._run(v, True)

    def apply_fwd_adj(self, q, v):
        """(Atilde q, Atilde^H v) for two device vectors of shape [n] and one dtype
        (skelfmm_apply_fwd_adj: one shared sweep for a real kernel in float32)."""
        torch = _torch()
        if q.dim() != 1 or v.dim() != 1 or q.shape[0] != self.n or v.shape[0] != self.n:
            raise ValueError("q and v must be vectors of length n")
        if q.dtype != v.dtype or not (q.is_cuda and v.is_cuda):
            raise ValueError("q and v must be device tensors of one dtype")
        q, v = q.contiguous(), v.contiguous()
        u, w = torch.empty_like(q), torch.empty_like(v)
        stream = torch.cuda.current_stream(q.device).cuda_stream
        _check(_lib.skelfmm_apply_fwd_adj(self._h, q.data_ptr(), v.data_ptr(), u.data_ptr(), w.data_ptr(),
                                          _dtype_code(q), stream))
        return u, w

    def autotune_fwd_adj(self) -> dict:
        """Time the two-column near field of the fused float32 forward + adjoint sweep
        with 1 .. 4 targets per lane; keep the fastest."""
        torch = _torch()
        chosen = ctypes.c_int32()
        ms = (ctypes.c_float * 4)()
        stream = torch.cuda.current_stream().cuda_stream
        _check(_lib.skelfmm_autotune_fwd_adj(self._h, stream, ctypes.byref(chosen), ms))
        return {"targets_per_lane": chosen.value, "ms": {t: ms[t - 1] for t in (1, 2, 3, 4)}}


def build(points, kind: str = "laplace", tol: float = 1e-6, leaf_size: int = 64, kappa: float = 0.0,
          proxy_shape: int = 0, proxy_points: int = 0, proxy_scale: float = 0.0, no_compression: bool = False,
          num_threads: int = 0, keep_transparent: bool = False, f64_leaf: bool = False,
          symmetric: bool = True, expansion: bool = True, compensated_leaf: bool = False,
          gpu_build: bool = False, f32_differences: bool = False) -> Operator:
    """Build the skeleton operator for ``points`` (n x dim, host, float64).

    ``symmetric=False`` evaluates both orders of every colleague pair separately
    (the pairing applies to the real Laplace kernels with one right-hand side);
    ``expansion=False`` keeps the float32 pair kernel on coordinate differences;
    ``compensated_leaf=True`` keeps its float32 partial sums to four products and
    forms its column sums in float64; ``gpu_build=True`` computes the
    interpolative decompositions on the current HIP device;
    ``f32_differences=True`` lets the float32 pair kernel form |d|^2 from float32
    coordinate differences in items whose reach is at most 1024 times their
    smallest point spacing."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    if pts.ndim != 2:
        raise ValueError("points must be n x dim")
    n, dim = pts.shape
    k = Kernel(HELMHOLTZ if kind == "helmholtz" else LAPLACE, dim, float(kappa))
    o = Options()
    o.proxy_shape, o.proxy_points, o.proxy_scale = proxy_shape, proxy_points, proxy_scale
    o.no_compression, o.num_threads = int(no_compression), num_threads
    o.keep_transparent, o.f64_leaf = int(keep_transparent), int(f64_leaf)
    o.nonsymmetric = int(not symmetric)
    o.no_expansion = int(not expansion)
    o.compensated_leaf = int(compensated_leaf)
    o.gpu_build = int(gpu_build)
    o.f32_differences = int(f32_differences)
    h = _vp()
    _check(_lib.skelfmm_build(pts.ctypes.data_as(_P(ctypes.c_double)), n, k, tol, leaf_size,
                              ctypes.byref(o), ctypes.byref(h)))
    return Operator(h, n, dim, k.kind)


class Batch:
    """Several operators applied together (one sweep per call)."""

    def __init__(self, ops):
        self.ops = list(ops)
        arr = (_vp * len(self.ops))(*[o.handle for o in self.ops])
        h = _vp()
        _check(_lib.skelfmm_batch_create(arr, len(self.ops), ctypes.byref(h)))
        self._h = h
        self._destroy = _lib.skelfmm_batch_destroy

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    def timing(self, enable: bool = True):
        """Enable (and zero) or disable per-pass HIP-event timing of eager batched sweeps."""
        _check(_lib.skelfmm_batch_timing(self._h, int(enable)))

    def timing_read(self) -> dict:
        ms = (ctypes.c_double * len(PASSES))()
        n = ctypes.c_int64()
        _check(_lib.skelfmm_batch_timing_read(self._h, ms, ctypes.byref(n)))
        out = {p: ms[i] for i, p in enumerate(PASSES)}
        out["sweeps"] = n.value
        return out

    def autotune_transfers(self, nrhs: int) -> dict:
        """Time the float32 many-RHS matrix-core transfers of the merged sweep; keep the fastest."""
        torch = _torch()
        chosen = ctypes.c_int32()
        ms = (ctypes.c_float * NXFER)()
        _check(_lib.skelfmm_batch_autotune_transfers(self._h, nrhs, torch.cuda.current_stream().cuda_stream,
                                                     ctypes.byref(chosen), ms))
        return {"shape": chosen.value, "ms": [ms[i] for i in range(NXFER)]}

    def apply(self, qs, adjoint: bool = False):
        """Outputs for every operator, each shaped like its input ([n] or [n, nrhs])."""
        torch = _torch()
        shapes = [q.shape for q in qs]
        qs = [q.reshape(q.shape[0], -1).contiguous() for q in qs]
        if len(qs) != len(self.ops) or any(q.shape[0] != o.n for q, o in zip(qs, self.ops)):
            raise ValueError("one input of matching length per operator")
        if len({q.shape[1] for q in qs}) != 1 or len({q.dtype for q in qs}) != 1:
            raise ValueError("batched inputs must share nrhs and dtype")
        us = [torch.empty_like(q) for q in qs]
        nrhs = qs[0].shape[1]
        qa = (_vp * len(qs))(*[q.data_ptr() for q in qs])
        ua = (_vp * len(us))(*[u.data_ptr() for u in us])
        stream = torch.cuda.current_stream(qs[0].device).cuda_stream
        _check(_lib.skelfmm_batch_apply(self._h, qa, ua, nrhs, _dtype_code(qs[0]), int(adjoint), stream))
        return [u.reshape(sh) for u, sh in zip(us, shapes)]


def _make_autograd():
    torch = _torch()

    class FmmApply(torch.autograd.Function):
        """u = Atilde q; backward gives dL/dq = Atilde^H (dL/du) via the adjoint sweep."""

        @staticmethod
        def forward(ctx, q, op):
            ctx.op = op
            return op.apply(q)

        @staticmethod
        def backward(ctx, grad_u):
            return ctx.op.apply_adjoint(grad_u.contiguous()), None

    return FmmApply


def _make_batch_autograd():
    torch = _torch()

    class BatchFmmApply(torch.autograd.Function):
        """[u_g] = [Atilde_g q_g] in one batched sweep; backward is one batched adjoint sweep."""

        @staticmethod
        def forward(ctx, batch, *qs):
            ctx.batch = batch
            return tuple(batch.apply(list(qs)))

        @staticmethod
        def backward(ctx, *grads):
            return (None, *ctx.batch.apply([g.contiguous() for g in grads], adjoint=True))

    return BatchFmmApply


_FmmApply = None
_BatchFmmApply = None


def batch_fmm_apply(batch: "Batch", qs):
    """Differentiable batched apply: one sweep forward, one adjoint sweep backward."""
    global _BatchFmmApply
    if _BatchFmmApply is None:
        _BatchFmmApply = _make_batch_autograd()
    return list(_BatchFmmApply.apply(batch, *qs))


def fmm_apply(op: Operator, q):
    """Differentiable apply: a torch.autograd.Function whose backward is the adjoint sweep."""
    global _FmmApply
    if _FmmApply is None:
        _FmmApply = _make_autograd()
    return _FmmApply.apply(q, op)
