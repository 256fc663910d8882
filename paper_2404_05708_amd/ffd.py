"""Thin Python binding of the C ABI in include/ffd.h (argument marshalling only).

Every computation happens in the HIP library ``libffd.so``; this module only
turns torch tensors (device memory, streams) and host offset arrays into the
pointers the C functions take.  If the library is not built, importing the
binding raises: there is no fallback path.

Functions keep the C names: ``ffd_distance``, ``ffd_distance_i32``,
``ffd_batch``, ``ffd_batch_i32``, ``ffd_cross``, ``ffd_cross_i32``,
``ffd_workspace_size``, ``ffd_set_scratch``, ``ffd_set_tuning``,
``ffd_create``, ``ffd_destroy``.  ``Context`` is a small convenience wrapper around them.
"""
import ctypes
import os

import numpy as np
import torch

# FFD_LIBRARY may name another build of the same library (e.g. a debug build)
LIB_PATH = os.environ.get("FFD_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                         "libffd.so")

FFD_OK = 0
FFD_E_INVALID = -1
FFD_E_UNSUPPORTED = -2
FFD_E_NOMEM = -3
FFD_E_DEVICE = -4
FFD_E_BUSY = -5
FFD_E_TIMEOUT = -6
FFD_E_CANCELED = -7
FFD_E_EXPIRED = -8
FFD_EUCLIDEAN = 0
FFD_SQEUCLIDEAN = 1
FFD_MANHATTAN = 2
FFD_CHEBYSHEV = 3
FFD_HAVERSINE = 4  # (latitude, longitude) in radians, dim 2; float32 Frechet calls only
FFD_OP_BATCH = 0
FFD_OP_CROSS = 1
FFD_OP_PAIR = 2
FFD_OP_DECIDE = 3
FFD_OP_KNN = 4
FFD_MAX_DIM = 16

EXPORTS = (
    "ffd_create", "ffd_create_planner", "ffd_destroy", "ffd_strerror", "ffd_last_error", "ffd_version",
    "ffd_distance", "ffd_distance_i32", "ffd_batch", "ffd_batch_i32", "ffd_cross",
    "ffd_cross_i32", "ffd_workspace_size", "ffd_set_tuning", "ffd_last_launch", "ffd_set_split", "ffd_last_errors",
    "ffd_set_kernel_timing", "ffd_kernel_time",
    "ffd_db_create", "ffd_db_destroy", "ffd_server_arena_size", "ffd_server_create", "ffd_server_destroy",
    "ffd_server_submit", "ffd_server_poll", "ffd_server_wait", "ffd_server_get_stats", "ffd_server_reset_stats",
    "ffd_server_last_error", "ffd_server_cancel", "ffd_server_set_deadline", "ffd_set_tune_cache",
    "ffd_autotune_batch",
    "ffd_autotune_cross",
    "ffd_dtw_distance", "ffd_dtw_distance_i32", "ffd_dtw_batch", "ffd_dtw_batch_i32", "ffd_dtw_cross",
    "ffd_dtw_cross_i32", "ffd_plan_describe", "ffd_levenshtein_distance", "ffd_levenshtein_batch",
    "ffd_levenshtein_cross", "ffd_decide_batch", "ffd_knn", "ffd_knn_batch", "ffd_last_search", "ffd_set_scratch",
    "ffd_batch_noalloc",
)


class SearchInfo(ctypes.Structure):
    _fields_ = [("exact", ctypes.c_int64), ("bounded", ctypes.c_int64), ("rejected", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class LaunchInfo(ctypes.Structure):
    _fields_ = [("rows_per_lane", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("lds_per_wave", ctypes.c_int32),
                ("exact", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("pipelined", ctypes.c_int32), ("helper_waves", ctypes.c_int32),
                ("stream_steps", ctypes.c_int64), ("per_lane", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class PlanSummary(ctypes.Structure):
    _fields_ = [("rows_per_lane", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("cooperative", ctypes.c_int32),
                ("rings", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("link_elems", ctypes.c_int64), ("stream_steps", ctypes.c_int64), ("jobs", ctypes.c_int64),
                ("pipelined", ctypes.c_int32), ("per_lane", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# one entry of a plan's job table (ffd_plan_job, 64 bytes)
PLAN_JOB = np.dtype([("out_base", "<i8"), ("link_in", "<i8"), ("link_out", "<i8"), ("row_sel", "<i4"),
                     ("row_idx", "<i4"), ("col_sel", "<i4"), ("col_first", "<i4"), ("col_count", "<i4"),
                     ("out_stride", "<i4"), ("band_first", "<i4"), ("band_count", "<i4"), ("flag_in", "<i4"),
                     ("flag_out", "<i4")])


class Tuning(ctypes.Structure):
    _fields_ = [("rows_per_lane", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32), ("split", ctypes.c_float),
                ("ms", ctypes.c_float), ("ms_planner", ctypes.c_float), ("tried", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("deferred", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("qps", ctypes.c_double), ("cells_per_s", ctypes.c_double),
                ("requests_per_launch", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("launches_by_rows", ctypes.c_int64 * 8), ("canceled", ctypes.c_int64),
                ("expired", ctypes.c_int64)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["launches_by_rows"] = list(d["launches_by_rows"])
        return d


class FFDError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


def _load(path=None):
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    sz = ctypes.c_size_t
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.ffd_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    lib.ffd_create.restype = ctypes.c_int
    lib.ffd_create_planner.argtypes = [i32, i64, ctypes.POINTER(vp)]
    lib.ffd_create_planner.restype = ctypes.c_int
    lib.ffd_destroy.argtypes = [vp]
    lib.ffd_destroy.restype = None
    lib.ffd_strerror.argtypes = [ctypes.c_int]
    lib.ffd_strerror.restype = ctypes.c_char_p
    lib.ffd_last_error.argtypes = [vp]
    lib.ffd_last_error.restype = ctypes.c_char_p
    lib.ffd_version.argtypes = []
    lib.ffd_version.restype = ctypes.c_char_p
    for name in ("ffd_distance", "ffd_distance_i32", "ffd_dtw_distance", "ffd_dtw_distance_i32"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, i64, vp, i64, i32, i32, vp, vp]
        fn.restype = ctypes.c_int
    for name in ("ffd_batch", "ffd_batch_i32", "ffd_dtw_batch", "ffd_dtw_batch_i32"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, i64p, vp, i64p, i64, i32, i32, vp, vp, sz, vp]
        fn.restype = ctypes.c_int
    for name in ("ffd_cross", "ffd_cross_i32", "ffd_dtw_cross", "ffd_dtw_cross_i32"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, i64p, i64, vp, i64p, i64, i32, i32, vp, vp, sz, vp]
        fn.restype = ctypes.c_int
    lib.ffd_workspace_size.argtypes = [vp, i32, i64p, i64, i64p, i64, i32, ctypes.POINTER(sz)]
    lib.ffd_workspace_size.restype = ctypes.c_int
    lib.ffd_batch_noalloc.argtypes = [vp, vp, i64p, vp, i64p, i64, i32, i32, vp, vp]
    lib.ffd_batch_noalloc.restype = ctypes.c_int
    lib.ffd_set_scratch.argtypes = [vp, vp, sz]
    lib.ffd_set_scratch.restype = ctypes.c_int
    lib.ffd_set_tuning.argtypes = [vp, i32, i32]
    lib.ffd_set_tuning.restype = ctypes.c_int
    lib.ffd_last_errors.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.ffd_last_errors.restype = ctypes.c_int
    lib.ffd_set_split.argtypes = [vp, ctypes.c_float]
    lib.ffd_set_split.restype = ctypes.c_int
    lib.ffd_last_launch.argtypes = [vp, ctypes.POINTER(LaunchInfo)]
    lib.ffd_last_launch.restype = ctypes.c_int
    lib.ffd_set_kernel_timing.argtypes = [vp, i32]
    lib.ffd_set_kernel_timing.restype = ctypes.c_int
    lib.ffd_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.ffd_kernel_time.restype = ctypes.c_int
    lib.ffd_levenshtein_distance.argtypes = [vp, vp, i64, vp, i64, i32, vp, vp]
    lib.ffd_levenshtein_distance.restype = ctypes.c_int
    lib.ffd_levenshtein_batch.argtypes = [vp, vp, i64p, vp, i64p, i64, i32, vp, vp, sz, vp]
    lib.ffd_levenshtein_batch.restype = ctypes.c_int
    lib.ffd_levenshtein_cross.argtypes = [vp, vp, i64p, i64, vp, i64p, i64, i32, vp, vp, sz, vp]
    lib.ffd_levenshtein_cross.restype = ctypes.c_int
    lib.ffd_plan_describe.argtypes = [vp, i32, i64p, i64, i64p, i64, i32, i32, i32, i32,
                                      ctypes.POINTER(PlanSummary), vp, i64, vp, i64]
    lib.ffd_plan_describe.restype = ctypes.c_int
    lib.ffd_autotune_batch.argtypes = [vp, vp, i64p, vp, i64p, i64, i32, i32, vp, vp, sz, vp, ctypes.POINTER(Tuning)]
    lib.ffd_autotune_batch.restype = ctypes.c_int
    lib.ffd_autotune_cross.argtypes = [vp, vp, i64p, i64, vp, i64p, i64, i32, i32, vp, vp, sz, vp,
                                       ctypes.POINTER(Tuning)]
    lib.ffd_autotune_cross.restype = ctypes.c_int
    lib.ffd_decide_batch.argtypes = [vp, vp, i64p, vp, i64p, i64, i32, i32, ctypes.c_float, vp, vp]
    lib.ffd_decide_batch.restype = ctypes.c_int
    lib.ffd_knn.argtypes = [vp, vp, i64, vp, i64p, i64, i32, i32, i32, vp, vp, vp]
    lib.ffd_knn.restype = ctypes.c_int
    lib.ffd_knn_batch.argtypes = [vp, vp, i64p, i64, vp, i64p, i64, i32, i32, i32, vp, vp, vp]
    lib.ffd_knn_batch.restype = ctypes.c_int
    lib.ffd_last_search.argtypes = [vp, ctypes.POINTER(SearchInfo)]
    lib.ffd_last_search.restype = ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.ffd_db_create.argtypes = [vp, vp, i64p, i64, i32, ctypes.POINTER(vp)]
    lib.ffd_db_create.restype = ctypes.c_int
    lib.ffd_db_destroy.argtypes = [vp]
    lib.ffd_db_destroy.restype = None
    lib.ffd_server_arena_size.argtypes = [vp, i32, i64, ctypes.POINTER(sz)]
    lib.ffd_server_arena_size.restype = ctypes.c_int
    lib.ffd_server_create.argtypes = [vp, vp, sz, i32, i64, ctypes.POINTER(vp)]
    lib.ffd_server_create.restype = ctypes.c_int
    lib.ffd_server_destroy.argtypes = [vp]
    lib.ffd_server_destroy.restype = None
    lib.ffd_server_submit.argtypes = [vp, vp, i64, i32, vp, u64p]
    lib.ffd_server_submit.restype = ctypes.c_int
    lib.ffd_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]
    lib.ffd_server_poll.restype = ctypes.c_int
    lib.ffd_server_wait.argtypes = [vp, ctypes.c_uint64, i64]
    lib.ffd_server_wait.restype = ctypes.c_int
    lib.ffd_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.ffd_server_get_stats.restype = ctypes.c_int
    lib.ffd_server_reset_stats.argtypes = [vp]
    lib.ffd_server_reset_stats.restype = ctypes.c_int
    lib.ffd_server_last_error.argtypes = [vp]
    lib.ffd_server_last_error.restype = ctypes.c_char_p
    lib.ffd_server_cancel.argtypes = [vp, ctypes.c_uint64]
    lib.ffd_server_cancel.restype = ctypes.c_int
    lib.ffd_server_set_deadline.argtypes = [vp, i64]
    lib.ffd_server_set_deadline.restype = ctypes.c_int
    lib.ffd_set_tune_cache.argtypes = [vp, ctypes.c_char_p]
    lib.ffd_set_tune_cache.restype = ctypes.c_int
    return lib


lib = _load()


def load_library(path):
    """Another build of the library (for example the debug variant the
    stress tests use), loaded beside the default one with the same
    signatures; its functions are called directly."""
    return _load(path)


def _check(rc, ctx=None):
    if rc != FFD_OK:
        msg = lib.ffd_strerror(rc).decode()
        if ctx:
            detail = lib.ffd_last_error(ctx).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise FFDError(rc, msg)


def _dev_ptr(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _curve(t, dtype, name):
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    if t.dim() != 2:
        raise ValueError(f"{name} must have shape (points, dim)")
    return t, _dev_ptr(t, dtype, name)


def _offsets(off):
    a = off.detach().cpu().numpy() if isinstance(off, torch.Tensor) else np.asarray(off)
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def ffd_version():
    return lib.ffd_version().decode()


def ffd_create(device=0):
    h = ctypes.c_void_p()
    _check(lib.ffd_create(int(device), ctypes.byref(h)))
    return h


def ffd_create_planner(compute_units=256, lds_per_block=160 * 1024):
    h = ctypes.c_void_p()
    _check(lib.ffd_create_planner(int(compute_units), int(lds_per_block), ctypes.byref(h)))
    return h


def ffd_destroy(ctx):
    lib.ffd_destroy(ctx)
    _MEM.pop(_key(ctx), None)


# Device memory the binding owns per context, for calls made without an
# explicit workspace and for the context's scratch (long single pairs, the
# search calls): torch tensors kept alive as long as the context, grown when
# a call reports FFD_E_NOMEM.  A temporary per call could be handed back by
# torch's caching allocator to other work while a kernel on another stream
# still uses it; memory held here cannot.
class _CtxMem:
    def __init__(self):
        self.ws = None
        self.scratch = None


_MEM = {}


def _key(ctx):
    return ctx.value if isinstance(ctx, ctypes.c_void_p) else int(ctx)


def _mem(ctx):
    return _MEM.setdefault(_key(ctx), _CtxMem())


def _grown(old, nbytes, device):
    """A tensor of at least nbytes on device; the old one (if any) is dropped
    only after the device has finished the work that may use it."""
    if old is not None:
        torch.cuda.synchronize(old.device)
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def ffd_set_scratch(ctx, scratch):
    """Register a uint8 device tensor (or None) as the context's scratch; the
    caller keeps it alive while it is registered."""
    if scratch is None:
        _check(lib.ffd_set_scratch(ctx, None, 0), ctx)
    else:
        _check(lib.ffd_set_scratch(ctx, _dev_ptr(scratch, torch.uint8, "scratch"), scratch.numel()), ctx)


def _with_scratch(ctx, device, size_fn, call):
    """Run call(); if it needs more scratch than the context has, grow the
    binding's scratch to size_fn() bytes, register it and run it again."""
    rc = call()
    if rc == FFD_E_NOMEM:
        mem = _mem(ctx)
        mem.scratch = _grown(mem.scratch, size_fn(), device)
        ffd_set_scratch(ctx, mem.scratch)
        rc = call()
    _check(rc, ctx)


def ffd_set_tuning(ctx, rows_per_lane=0, waves_per_simd=0):
    _check(lib.ffd_set_tuning(ctx, int(rows_per_lane), int(waves_per_simd)), ctx)


def ffd_last_errors(ctx):
    v = ctypes.c_int32()
    _check(lib.ffd_last_errors(ctx, ctypes.byref(v)), ctx)
    return v.value


def ffd_set_tune_cache(ctx, path):
    _check(lib.ffd_set_tune_cache(ctx, None if path is None else os.fsencode(path)), ctx)


def ffd_set_split(ctx, share=0.0):
    _check(lib.ffd_set_split(ctx, float(share)), ctx)


def ffd_decide_batch(ctx, P, p_off, Q, q_off, eps, metric=FFD_EUCLIDEAN, out=None, stream=None):
    """Decider (early abandoning): out[k] = delta_k if delta_k <= eps, else +inf."""
    P, Pp = _curve(P, torch.float32, "P")
    Q, Qp = _curve(Q, torch.float32, "Q")
    if P.shape[1] != Q.shape[1]:
        raise ValueError("P and Q must have the same dimension")
    po, pop = _offsets(p_off)
    qo, qop = _offsets(q_off)
    npairs = len(po) - 1
    if len(qo) - 1 != npairs:
        raise ValueError("p_off and q_off must describe the same number of pairs")
    if out is None:
        out = torch.empty(max(npairs, 1), dtype=torch.float32, device=P.device)
    outp = _dev_ptr(out, torch.float32, "out")
    _with_scratch(ctx, P.device, lambda: ffd_workspace_size(ctx, FFD_OP_DECIDE, po, qo, P.shape[1]),
                  lambda: lib.ffd_decide_batch(ctx, Pp, pop, Qp, qop, npairs, P.shape[1], int(metric), float(eps),
                                               outp, _stream(stream)))
    return out[:npairs]


def ffd_knn(ctx, q, DB, db_off, k, metric=FFD_EUCLIDEAN, stream=None):
    """The k database curves nearest to q: (int64 indices, float32 distances),
    device tensors of k entries (index -1 / +inf past the database size)."""
    q, qp = _curve(q, torch.float32, "q")
    DB, Dp = _curve(DB, torch.float32, "DB")
    if q.shape[1] != DB.shape[1]:
        raise ValueError("q and DB must have the same dimension")
    do, dop = _offsets(db_off)
    idx = torch.empty(max(int(k), 1), dtype=torch.int64, device=q.device)
    dist = torch.empty(max(int(k), 1), dtype=torch.float32, device=q.device)
    ip, dp = _dev_ptr(idx, torch.int64, "idx"), _dev_ptr(dist, torch.float32, "dist")
    _with_scratch(ctx, q.device, lambda: ffd_workspace_size(ctx, FFD_OP_KNN, [0, q.shape[0]], do, q.shape[1]),
                  lambda: lib.ffd_knn(ctx, qp, q.shape[0], Dp, dop, len(do) - 1, q.shape[1], int(metric), int(k),
                                      ip, dp, _stream(stream)))
    return idx[:k], dist[:k]


def ffd_knn_batch(ctx, Q, q_off, DB, db_off, k, metric=FFD_EUCLIDEAN, stream=None):
    """k nearest database curves of each of nq queries (CSR): (int64
    indices, float32 distances), device tensors of shape (nq, k)."""
    Q, Qp = _curve(Q, torch.float32, "Q")
    DB, Dp = _curve(DB, torch.float32, "DB")
    if Q.shape[1] != DB.shape[1]:
        raise ValueError("Q and DB must have the same dimension")
    qo, qop = _offsets(q_off)
    do, dop = _offsets(db_off)
    nq, k = len(qo) - 1, int(k)
    idx = torch.empty((max(nq, 1), max(k, 1)), dtype=torch.int64, device=Q.device)
    dist = torch.empty((max(nq, 1), max(k, 1)), dtype=torch.float32, device=Q.device)
    ip, dp = _dev_ptr(idx, torch.int64, "idx"), _dev_ptr(dist, torch.float32, "dist")
    _with_scratch(ctx, Q.device, lambda: ffd_workspace_size(ctx, FFD_OP_KNN, qo, do, Q.shape[1]),
                  lambda: lib.ffd_knn_batch(ctx, Qp, qop, nq, Dp, dop, len(do) - 1, Q.shape[1], int(metric), k,
                                            ip, dp, _stream(stream)))
    return idx[:nq, :k], dist[:nq, :k]


def ffd_last_search(ctx):
    info = SearchInfo()
    _check(lib.ffd_last_search(ctx, ctypes.byref(info)), ctx)
    return info.as_dict()


def ffd_last_launch(ctx):
    info = LaunchInfo()
    _check(lib.ffd_last_launch(ctx, ctypes.byref(info)), ctx)
    return info.as_dict()


def ffd_set_kernel_timing(ctx, enable):
    _check(lib.ffd_set_kernel_timing(ctx, 1 if enable else 0), ctx)


def ffd_kernel_time(ctx):
    """(summed kernel milliseconds, launches) recorded since the last read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib.ffd_kernel_time(ctx, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


def _pair(fn, dtype, odtype, ctx, p, q, metric, out, stream):
    p, pp = _curve(p, dtype, "p")
    q, qp = _curve(q, dtype, "q")
    if p.shape[1] != q.shape[1]:
        raise ValueError("p and q must have the same dimension")
    if out is None:
        out = torch.empty(1, dtype=odtype, device=p.device)
    outp = _dev_ptr(out, odtype, "out")
    _with_scratch(ctx, p.device, lambda: ffd_workspace_size(ctx, FFD_OP_PAIR, [0, p.shape[0]], [0, q.shape[0]],
                                                            p.shape[1]),
                  lambda: fn(ctx, pp, p.shape[0], qp, q.shape[0], p.shape[1], int(metric), outp, _stream(stream)))
    return out


def ffd_distance(ctx, p, q, metric=FFD_EUCLIDEAN, out=None, stream=None):
    return _pair(lib.ffd_distance, torch.float32, torch.float32, ctx, p, q, metric, out, stream)


def ffd_distance_i32(ctx, p, q, metric=FFD_SQEUCLIDEAN, out=None, stream=None):
    return _pair(lib.ffd_distance_i32, torch.int32, torch.int64, ctx, p, q, metric, out, stream)


def ffd_dtw_distance(ctx, p, q, metric=FFD_EUCLIDEAN, out=None, stream=None):
    return _pair(lib.ffd_dtw_distance, torch.float32, torch.float32, ctx, p, q, metric, out, stream)


def ffd_dtw_distance_i32(ctx, p, q, metric=FFD_SQEUCLIDEAN, out=None, stream=None):
    return _pair(lib.ffd_dtw_distance_i32, torch.int32, torch.int64, ctx, p, q, metric, out, stream)


def ffd_levenshtein_distance(ctx, p, q, out=None, stream=None):
    p, pp = _curve(p, torch.int32, "p")
    q, qp = _curve(q, torch.int32, "q")
    if p.shape[1] != q.shape[1]:
        raise ValueError("p and q must have the same dimension")
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=p.device)
    outp = _dev_ptr(out, torch.int64, "out")
    _with_scratch(ctx, p.device, lambda: ffd_workspace_size(ctx, FFD_OP_PAIR, [0, p.shape[0]], [0, q.shape[0]],
                                                            p.shape[1]),
                  lambda: lib.ffd_levenshtein_distance(ctx, pp, p.shape[0], qp, q.shape[0], p.shape[1], outp,
                                                       _stream(stream)))
    return out


def ffd_levenshtein_batch(ctx, P, p_off, Q, q_off, out=None, workspace=None, stream=None):
    P, Pp = _curve(P, torch.int32, "P")
    Q, Qp = _curve(Q, torch.int32, "Q")
    if P.shape[1] != Q.shape[1]:
        raise ValueError("P and Q must have the same dimension")
    po, pop = _offsets(p_off)
    qo, qop = _offsets(q_off)
    npairs = len(po) - 1
    if len(qo) - 1 != npairs:
        raise ValueError("p_off and q_off must describe the same number of pairs")
    if out is None:
        out = torch.empty(max(npairs, 1), dtype=torch.int64, device=P.device)
    _run_ws(ctx, FFD_OP_BATCH, po, qo, P.shape[1], P.device, workspace,
            lambda wsp, wsn: lib.ffd_levenshtein_batch(ctx, Pp, pop, Qp, qop, npairs, P.shape[1],
                                                       _dev_ptr(out, torch.int64, "out"), wsp, wsn,
                                                       _stream(stream)))
    return out[:npairs]


def ffd_levenshtein_cross(ctx, Qs, q_off, DB, db_off, out=None, workspace=None, stream=None):
    Qs, Qp = _curve(Qs, torch.int32, "Qs")
    DB, Dp = _curve(DB, torch.int32, "DB")
    if Qs.shape[1] != DB.shape[1]:
        raise ValueError("Qs and DB must have the same dimension")
    qo, qop = _offsets(q_off)
    do, dop = _offsets(db_off)
    nq, ndb = len(qo) - 1, len(do) - 1
    if out is None:
        out = torch.empty(max(nq * ndb, 1), dtype=torch.int64, device=Qs.device)
    _run_ws(ctx, FFD_OP_CROSS, qo, do, Qs.shape[1], Qs.device, workspace,
            lambda wsp, wsn: lib.ffd_levenshtein_cross(ctx, Qp, qop, nq, Dp, dop, ndb, Qs.shape[1],
                                                       _dev_ptr(out, torch.int64, "out"), wsp, wsn,
                                                       _stream(stream)))
    return out[:nq * ndb].reshape(nq, ndb)


def ffd_plan_describe(ctx, op, a_off, b_off, dim, exact=False, dtw=False, metric=FFD_EUCLIDEAN,
                      levenshtein=False):
    """The plan a call would launch: (summary dict, job table as a PLAN_JOB
    array, first job of each wave as int32[waves + 1]).  Host-only."""
    measure = 2 if levenshtein else (1 if dtw else 0)
    ao, aop = _offsets(a_off)
    bo, bop = _offsets(b_off)
    sm = PlanSummary()
    args = (ctx, int(op), aop, len(ao) - 1, bop, len(bo) - 1, int(dim), int(bool(exact)), measure,
            int(metric), ctypes.byref(sm))
    _check(lib.ffd_plan_describe(*args, None, 0, None, 0), ctx)
    jobs = np.zeros(sm.jobs, dtype=PLAN_JOB)
    wj = np.zeros(sm.waves + 1, dtype=np.int32)
    _check(lib.ffd_plan_describe(*args, ctypes.c_void_p(jobs.ctypes.data), len(jobs),
                                 ctypes.c_void_p(wj.ctypes.data), len(wj)), ctx)
    return sm.as_dict(), jobs, wj


def ffd_workspace_size(ctx, op, a_off, b_off, dim):
    a, ap = _offsets(a_off)
    b, bp = _offsets(b_off)
    n = ctypes.c_size_t()
    _check(lib.ffd_workspace_size(ctx, int(op), ap, len(a) - 1, bp, len(b) - 1, int(dim),
                                  ctypes.byref(n)), ctx)
    return n.value


def _run_ws(ctx, op, a_off, b_off, dim, device, workspace, call, presize=False):
    """call(workspace pointer, bytes) with the caller's workspace, or with
    the context's own one (grown to ffd_workspace_size when the call reports
    FFD_E_NOMEM, or before the call with `presize`) when the caller gives
    none."""
    if workspace is not None:
        _check(call(_dev_ptr(workspace, workspace.dtype, "workspace"),
                    workspace.numel() * workspace.element_size()), ctx)
        return
    mem = _mem(ctx)
    if mem.ws is not None and mem.ws.device == device and not presize:
        rc = call(ctypes.c_void_p(mem.ws.data_ptr()), mem.ws.numel())
        if rc != FFD_E_NOMEM:
            _check(rc, ctx)
            return
    mem.ws = _grown(mem.ws, ffd_workspace_size(ctx, op, a_off, b_off, dim), device)
    _check(call(ctypes.c_void_p(mem.ws.data_ptr()), mem.ws.numel()), ctx)


def _batch(fn, dtype, odtype, ctx, P, p_off, Q, q_off, metric, out, workspace, stream):
    P, Pp = _curve(P, dtype, "P")
    Q, Qp = _curve(Q, dtype, "Q")
    if P.shape[1] != Q.shape[1]:
        raise ValueError("P and Q must have the same dimension")
    po, pop = _offsets(p_off)
    qo, qop = _offsets(q_off)
    npairs = len(po) - 1
    if len(qo) - 1 != npairs:
        raise ValueError("p_off and q_off must describe the same number of pairs")
    if out is None:
        out = torch.empty(max(npairs, 1), dtype=odtype, device=P.device)
    _run_ws(ctx, FFD_OP_BATCH, po, qo, P.shape[1], P.device, workspace,
            lambda wsp, wsn: fn(ctx, Pp, pop, Qp, qop, npairs, P.shape[1], int(metric),
                                _dev_ptr(out, odtype, "out"), wsp, wsn, _stream(stream)))
    return out[:npairs]


def ffd_batch(ctx, P, p_off, Q, q_off, metric=FFD_EUCLIDEAN, out=None, workspace=None, stream=None):
    return _batch(lib.ffd_batch, torch.float32, torch.float32, ctx, P, p_off, Q, q_off, metric,
                  out, workspace, stream)


def ffd_batch_noalloc(ctx, P, p_off, Q, q_off, metric=FFD_EUCLIDEAN, out=None, stream=None):
    """ffd_batch with the library's static device scratch: no workspace, no
    device allocation by the library (out is allocated here when not given)."""
    P, Pp = _curve(P, torch.float32, "P")
    Q, Qp = _curve(Q, torch.float32, "Q")
    if P.shape[1] != Q.shape[1]:
        raise ValueError("P and Q must have the same dimension")
    po, pop = _offsets(p_off)
    qo, qop = _offsets(q_off)
    npairs = len(po) - 1
    if len(qo) - 1 != npairs:
        raise ValueError("p_off and q_off must describe the same number of pairs")
    if out is None:
        out = torch.empty(max(npairs, 1), dtype=torch.float32, device=P.device)
    _check(lib.ffd_batch_noalloc(ctx, Pp, pop, Qp, qop, npairs, P.shape[1], int(metric),
                                 _dev_ptr(out, torch.float32, "out"), _stream(stream)), ctx)
    return out[:npairs]


def ffd_batch_i32(ctx, P, p_off, Q, q_off, metric=FFD_SQEUCLIDEAN, out=None, workspace=None,
                  stream=None):
    return _batch(lib.ffd_batch_i32, torch.int32, torch.int64, ctx, P, p_off, Q, q_off, metric,
                  out, workspace, stream)


def ffd_dtw_batch(ctx, P, p_off, Q, q_off, metric=FFD_EUCLIDEAN, out=None, workspace=None, stream=None):
    return _batch(lib.ffd_dtw_batch, torch.float32, torch.float32, ctx, P, p_off, Q, q_off, metric,
                  out, workspace, stream)


def ffd_dtw_batch_i32(ctx, P, p_off, Q, q_off, metric=FFD_SQEUCLIDEAN, out=None, workspace=None,
                      stream=None):
    return _batch(lib.ffd_dtw_batch_i32, torch.int32, torch.int64, ctx, P, p_off, Q, q_off, metric,
                  out, workspace, stream)


def _cross(fn, dtype, odtype, ctx, Qs, q_off, DB, db_off, metric, out, workspace, stream):
    Qs, Qp = _curve(Qs, dtype, "Qs")
    DB, Dp = _curve(DB, dtype, "DB")
    if Qs.shape[1] != DB.shape[1]:
        raise ValueError("Qs and DB must have the same dimension")
    qo, qop = _offsets(q_off)
    do, dop = _offsets(db_off)
    nq, ndb = len(qo) - 1, len(do) - 1
    if out is None:
        out = torch.empty(max(nq * ndb, 1), dtype=odtype, device=Qs.device)
    _run_ws(ctx, FFD_OP_CROSS, qo, do, Qs.shape[1], Qs.device, workspace,
            lambda wsp, wsn: fn(ctx, Qp, qop, nq, Dp, dop, ndb, Qs.shape[1], int(metric),
                                _dev_ptr(out, odtype, "out"), wsp, wsn, _stream(stream)))
    return out[:nq * ndb].reshape(nq, ndb)


def ffd_cross(ctx, Qs, q_off, DB, db_off, metric=FFD_EUCLIDEAN, out=None, workspace=None,
              stream=None):
    return _cross(lib.ffd_cross, torch.float32, torch.float32, ctx, Qs, q_off, DB, db_off, metric,
                  out, workspace, stream)


def ffd_cross_i32(ctx, Qs, q_off, DB, db_off, metric=FFD_SQEUCLIDEAN, out=None, workspace=None,
                  stream=None):
    return _cross(lib.ffd_cross_i32, torch.int32, torch.int64, ctx, Qs, q_off, DB, db_off, metric,
                  out, workspace, stream)


def ffd_dtw_cross(ctx, Qs, q_off, DB, db_off, metric=FFD_EUCLIDEAN, out=None, workspace=None,
                  stream=None):
    return _cross(lib.ffd_dtw_cross, torch.float32, torch.float32, ctx, Qs, q_off, DB, db_off, metric,
                  out, workspace, stream)


def ffd_dtw_cross_i32(ctx, Qs, q_off, DB, db_off, metric=FFD_SQEUCLIDEAN, out=None, workspace=None,
                      stream=None):
    return _cross(lib.ffd_dtw_cross_i32, torch.int32, torch.int64, ctx, Qs, q_off, DB, db_off, metric,
                  out, workspace, stream)


def ffd_autotune_batch(ctx, P, p_off, Q, q_off, metric=FFD_EUCLIDEAN, out=None, workspace=None, stream=None):
    """Time the launch shapes on this batch and keep the fastest for its offsets."""
    P, Pp = _curve(P, torch.float32, "P")
    Q, Qp = _curve(Q, torch.float32, "Q")
    po, pop = _offsets(p_off)
    qo, qop = _offsets(q_off)
    npairs = len(po) - 1
    if out is None:
        out = torch.empty(max(npairs, 1), dtype=torch.float32, device=P.device)
    t = Tuning()
    _run_ws(ctx, FFD_OP_BATCH, po, qo, P.shape[1], P.device, workspace,
            lambda wsp, wsn: lib.ffd_autotune_batch(ctx, Pp, pop, Qp, qop, npairs, P.shape[1], int(metric),
                                                    _dev_ptr(out, torch.float32, "out"), wsp, wsn,
                                                    _stream(stream), ctypes.byref(t)),
            presize=True)
    return t.as_dict()


def ffd_autotune_cross(ctx, Qs, q_off, DB, db_off, metric=FFD_EUCLIDEAN, out=None, workspace=None, stream=None):
    """Time the launch shapes on this query set x database and keep the fastest."""
    Qs, Qp = _curve(Qs, torch.float32, "Qs")
    DB, Dp = _curve(DB, torch.float32, "DB")
    qo, qop = _offsets(q_off)
    do, dop = _offsets(db_off)
    nq, ndb = len(qo) - 1, len(do) - 1
    if out is None:
        out = torch.empty(max(nq * ndb, 1), dtype=torch.float32, device=Qs.device)
    t = Tuning()
    _run_ws(ctx, FFD_OP_CROSS, qo, do, Qs.shape[1], Qs.device, workspace,
            lambda wsp, wsn: lib.ffd_autotune_cross(ctx, Qp, qop, nq, Dp, dop, ndb, Qs.shape[1], int(metric),
                                                    _dev_ptr(out, torch.float32, "out"), wsp, wsn,
                                                    _stream(stream), ctypes.byref(t)),
            presize=True)
    return t.as_dict()


class Context:
    """Owns one ffd_ctx; methods call the functions above."""

    def __init__(self, device=0):
        self.device = device
        self.handle = ffd_create(device)

    def close(self):
        if self.handle:
            ffd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tune_cache(self, path):
        ffd_set_tune_cache(self.handle, path)

    def set_tuning(self, rows_per_lane=0, waves_per_simd=0):
        ffd_set_tuning(self.handle, rows_per_lane, waves_per_simd)

    def last_errors(self):
        return ffd_last_errors(self.handle)

    def set_split(self, share=0.0):
        ffd_set_split(self.handle, share)

    def last_launch(self):
        return ffd_last_launch(self.handle)

    def set_kernel_timing(self, enable):
        ffd_set_kernel_timing(self.handle, enable)

    def kernel_time(self):
        return ffd_kernel_time(self.handle)

    def distance(self, p, q, metric=FFD_EUCLIDEAN, **kw):
        return ffd_distance(self.handle, p, q, metric, **kw)

    def distance_i32(self, p, q, metric=FFD_SQEUCLIDEAN, **kw):
        return ffd_distance_i32(self.handle, p, q, metric, **kw)

    def batch(self, P, p_off, Q, q_off, metric=FFD_EUCLIDEAN, **kw):
        return ffd_batch(self.handle, P, p_off, Q, q_off, metric, **kw)

    def batch_noalloc(self, P, p_off, Q, q_off, metric=FFD_EUCLIDEAN, **kw):
        return ffd_batch_noalloc(self.handle, P, p_off, Q, q_off, metric, **kw)

    def batch_i32(self, P, p_off, Q, q_off, metric=FFD_SQEUCLIDEAN, **kw):
        return ffd_batch_i32(self.handle, P, p_off, Q, q_off, metric, **kw)

    def cross(self, Qs, q_off, DB, db_off, metric=FFD_EUCLIDEAN, **kw):
        return ffd_cross(self.handle, Qs, q_off, DB, db_off, metric, **kw)

    def cross_i32(self, Qs, q_off, DB, db_off, metric=FFD_SQEUCLIDEAN, **kw):
        return ffd_cross_i32(self.handle, Qs, q_off, DB, db_off, metric, **kw)

    def dtw_distance(self, p, q, metric=FFD_EUCLIDEAN, **kw):
        return ffd_dtw_distance(self.handle, p, q, metric, **kw)

    def dtw_distance_i32(self, p, q, metric=FFD_SQEUCLIDEAN, **kw):
        return ffd_dtw_distance_i32(self.handle, p, q, metric, **kw)

    def dtw_batch(self, P, p_off, Q, q_off, metric=FFD_EUCLIDEAN, **kw):
        return ffd_dtw_batch(self.handle, P, p_off, Q, q_off, metric, **kw)

    def dtw_batch_i32(self, P, p_off, Q, q_off, metric=FFD_SQEUCLIDEAN, **kw):
        return ffd_dtw_batch_i32(self.handle, P, p_off, Q, q_off, metric, **kw)

    def dtw_cross(self, Qs, q_off, DB, db_off, metric=FFD_EUCLIDEAN, **kw):
        return ffd_dtw_cross(self.handle, Qs, q_off, DB, db_off, metric, **kw)

    def dtw_cross_i32(self, Qs, q_off, DB, db_off, metric=FFD_SQEUCLIDEAN, **kw):
        return ffd_dtw_cross_i32(self.handle, Qs, q_off, DB, db_off, metric, **kw)

    def levenshtein(self, p, q, **kw):
        return ffd_levenshtein_distance(self.handle, p, q, **kw)

    def decide_batch(self, P, p_off, Q, q_off, eps, metric=FFD_EUCLIDEAN, **kw):
        return ffd_decide_batch(self.handle, P, p_off, Q, q_off, eps, metric, **kw)

    def knn(self, q, DB, db_off, k, metric=FFD_EUCLIDEAN, **kw):
        return ffd_knn(self.handle, q, DB, db_off, k, metric, **kw)

    def knn_batch(self, Q, q_off, DB, db_off, k, metric=FFD_EUCLIDEAN, **kw):
        return ffd_knn_batch(self.handle, Q, q_off, DB, db_off, k, metric, **kw)

    def last_search(self):
        return ffd_last_search(self.handle)

    def levenshtein_batch(self, P, p_off, Q, q_off, **kw):
        return ffd_levenshtein_batch(self.handle, P, p_off, Q, q_off, **kw)

    def levenshtein_cross(self, Qs, q_off, DB, db_off, **kw):
        return ffd_levenshtein_cross(self.handle, Qs, q_off, DB, db_off, **kw)

    def autotune_batch(self, P, p_off, Q, q_off, metric=FFD_EUCLIDEAN, **kw):
        return ffd_autotune_batch(self.handle, P, p_off, Q, q_off, metric, **kw)

    def autotune_cross(self, Qs, q_off, DB, db_off, metric=FFD_EUCLIDEAN, **kw):
        return ffd_autotune_cross(self.handle, Qs, q_off, DB, db_off, metric, **kw)

    def workspace_size(self, op, a_off, b_off, dim):
        return ffd_workspace_size(self.handle, op, a_off, b_off, dim)

    def set_scratch(self, scratch):
        """Register caller device memory (uint8 tensor, kept alive by the
        caller) as the scratch; None returns to the binding's own."""
        ffd_set_scratch(self.handle, scratch)
        if scratch is None:
            _mem(self.handle).scratch = None


# ------------------------------------------------------------------ serving

class Database:
    """A device-resident database of float32 curves (ffd_db).  Keeps the
    coordinate tensor alive for as long as the handle exists."""

    def __init__(self, ctx, DB, db_off):
        DB, Dp = _curve(DB, torch.float32, "DB")
        do, dop = _offsets(db_off)
        self.ctx = ctx
        self.tensor = DB
        self.offsets = do
        self.ndb = len(do) - 1
        self.dim = DB.shape[1]
        h = ctypes.c_void_p()
        _check(lib.ffd_db_create(ctx.handle, Dp, dop, self.ndb, self.dim, ctypes.byref(h)), ctx.handle)
        self.handle = h

    def close(self):
        if self.handle:
            lib.ffd_db_destroy(self.handle)
            self.handle = None


class Server:
    """Continuous-batching query server over a Database (ffd_server).  The
    arena is a torch tensor on the database's device."""

    def __init__(self, db, max_slots=8, max_query=8192):
        self.db = db
        n = ctypes.c_size_t()
        _check(lib.ffd_server_arena_size(db.handle, int(max_slots), int(max_query), ctypes.byref(n)),
               db.ctx.handle)
        self.arena = torch.empty(max(n.value, 1), dtype=torch.uint8, device=db.tensor.device)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(lib.ffd_server_create(db.handle, ctypes.c_void_p(self.arena.data_ptr()), self.arena.numel(),
                                     int(max_slots), int(max_query), ctypes.byref(h)), db.ctx.handle)
        self.handle = h
        self._live = {}  # ticket -> (query copy, result array) kept alive until collected

    def _check(self, rc):
        if rc != FFD_OK:
            raise FFDError(rc, f"{lib.ffd_strerror(rc).decode()}: {lib.ffd_server_last_error(self.handle).decode()}")

    def submit(self, q, metric=FFD_EUCLIDEAN, out=None):
        """Submit a (n, dim) float32 host array; returns a ticket.  `out` (a
        float32 array of ndb entries) receives the results, a new one if
        None."""
        q = np.ascontiguousarray(q, dtype=np.float32)
        if q.ndim == 1:
            q = q.reshape(-1, 1)
        if q.shape[1] != self.db.dim:
            raise ValueError("query dimension differs from the database's")
        if out is None:
            out = np.empty(self.db.ndb, dtype=np.float32)
        elif out.dtype != np.float32 or out.shape != (self.db.ndb,) or not out.flags.c_contiguous:
            raise ValueError("out must be a contiguous float32 array of ndb entries")
        t = ctypes.c_uint64()
        self._check(lib.ffd_server_submit(self.handle, q.ctypes.data_as(ctypes.c_void_p), q.shape[0],
                                          int(metric), out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t)))
        self._live[t.value] = (q, out)
        return t.value

    def poll(self, ticket):
        """The result array once the request has finished, else None; a
        failed, canceled or expired request raises FFDError (its ticket is
        collected)."""
        done = ctypes.c_int32()
        rc = lib.ffd_server_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(done))
        if rc != FFD_OK:
            self._live.pop(ticket, None)
            self._check(rc)
        if not done.value:
            return None
        return self._live.pop(ticket)[1]

    def wait(self, ticket, timeout_us=-1):
        rc = lib.ffd_server_wait(self.handle, ctypes.c_uint64(ticket), int(timeout_us))
        if rc not in (FFD_OK, FFD_E_TIMEOUT):  # a timed-out wait leaves the ticket uncollected
            self._live.pop(ticket, None)
        self._check(rc)
        return self._live.pop(ticket)[1]

    def cancel(self, ticket):
        self._check(lib.ffd_server_cancel(self.handle, ctypes.c_uint64(ticket)))

    def set_deadline(self, timeout_us):
        self._check(lib.ffd_server_set_deadline(self.handle, int(timeout_us)))

    def stats(self):
        st = ServerStats()
        self._check(lib.ffd_server_get_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def reset_stats(self):
        self._check(lib.ffd_server_reset_stats(self.handle))

    def close(self):
        if self.handle:
            lib.ffd_server_destroy(self.handle)
            self.handle = None
            self._live.clear()
