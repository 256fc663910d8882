"""Plain CPU oracle for the discrete Frechet distance.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of ``bench.py`` may import this package.  The GPU library never
imports, links or calls it, and it imports nothing from the GPU library.

Contents
--------
* ``ffd_oracle.c`` (built into ``libffd_oracle.so``): FP64 memoised recursion
  (Algorithm 1), full-table iteration (Algorithm 3), the rolling two-row form
  of Algorithm 3 (Sec. 3, proof of Theorem 1: only two adjacent rows are
  live), exact int64 squared distances, a float32 replica of one fixed
  evaluation order, and a thread pool for many pairs.
* ``brute.py``: minimum over all monotone couplings (the Eiter--Mannila
  definition the paper builds on in Sec. 2), pure Python, tiny inputs only.
* ``paper_forms.py``: the paper's branch-free forms (Algorithms 2, 4 and 5
  with the scan and fold operators of Appendix A) in FP64 numpy, and the
  DTW algorithm of Appendix B (Algorithm B.1) in the same style.
* DTW (Appendix B): the table recurrence with the outer max replaced by a
  sum, M_ij = min{M_{i-1,j}, M_{i-1,j-1}, M_{i,j-1}} + d_ij, in FP64, exact
  int64, and a float32 replica (``dtw_*``).

* ``decide`` and ``knn``: the decider's and the k-nearest search's answers
  from a vector of distances (a comparison, and a sort by (distance, index)).

Inputs are float32 (widened exactly to FP64 inside) or int32 arrays of shape
(n, D), row-major.  Metric 0 = Euclidean (sqrt of the sum of squares per
cell), 1 = squared Euclidean, 2 = Manhattan (sum of |p_k - q_k|), 3 =
Chebyshev (max of |p_k - q_k|); int32 inputs take 1, 2 or 3.
"""
import ctypes
import os

import numpy as np

from .build_oracle import LIB as _LIB_PATH, build as _build

EUCLIDEAN = 0
SQEUCLIDEAN = 1
MANHATTAN = 2
CHEBYSHEV = 3
HAVERSINE = 4  # (latitude, longitude) in radians, dim 2; float inputs only

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            _build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        for name in ("ffdo_recursive", "ffdo_table", "ffdo_rolling"):
            fn = getattr(lib, name)
            fn.argtypes = [f32p, i64, f32p, i64, ci, ci, f64p]
            fn.restype = ci
        lib.ffdo_table_full.argtypes = [f32p, i64, f32p, i64, ci, ci, f64p]
        lib.ffdo_table_full.restype = ci
        lib.ffdo_rolling_state.argtypes = [f32p, i64, f32p, i64, ci, ci, f64p]
        lib.ffdo_rolling_state.restype = ci
        lib.ffdo_rolling_resume.argtypes = [f32p, i64, i64, f32p, i64, ci, ci, f64p, f64p]
        lib.ffdo_rolling_resume.restype = ci
        lib.ffdo_i32.argtypes = [i32p, i64, i32p, i64, ci, ci, i64p]
        lib.ffdo_i32.restype = ci
        lib.ffdo_f32_replica.argtypes = [f32p, i64, f32p, i64, ci, ci, f32p]
        lib.ffdo_f32_replica.restype = ci
        lib.ffdo_pairs.argtypes = [f32p, i64p, i64p, f32p, i64p, i64p, i64, ci, ci, i64p, ci, f64p]
        lib.ffdo_pairs.restype = ci
        lib.ffdo_pairs_i32.argtypes = [i32p, i64p, i64p, i32p, i64p, i64p, i64, ci, ci, i64p, ci, i64p]
        lib.ffdo_pairs_i32.restype = ci
        lib.ffdo_dtw.argtypes = [f32p, i64, f32p, i64, ci, ci, f64p]
        lib.ffdo_dtw.restype = ci
        lib.ffdo_dtw_i32.argtypes = [i32p, i64, i32p, i64, ci, ci, i64p]
        lib.ffdo_dtw_i32.restype = ci
        lib.ffdo_dtw_f32_replica.argtypes = [f32p, i64, f32p, i64, ci, ci, f32p]
        lib.ffdo_dtw_f32_replica.restype = ci
        lib.ffdo_dtw_pairs.argtypes = [f32p, i64p, i64p, f32p, i64p, i64p, i64, ci, ci, i64p, ci, f64p]
        lib.ffdo_dtw_pairs.restype = ci
        lib.ffdo_dtw_pairs_i32.argtypes = [i32p, i64p, i64p, i32p, i64p, i64p, i64, ci, ci, i64p, ci, i64p]
        lib.ffdo_dtw_pairs_i32.restype = ci
        lib.ffdo_lev.argtypes = [i32p, i64, i32p, i64, ci, i64p]
        lib.ffdo_lev.restype = ci
        lib.ffdo_lev_pairs.argtypes = [i32p, i64p, i64p, i32p, i64p, i64p, i64, ci, i64p, ci, i64p]
        lib.ffdo_lev_pairs.restype = ci
        lib.ffdo_now.argtypes = []
        lib.ffdo_now.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _curve_f32(x):
    a = np.ascontiguousarray(x, dtype=np.float32)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    if a.ndim != 2:
        raise ValueError("curve must have shape (n, D)")
    return a


def _curve_i32(x):
    a = np.ascontiguousarray(x, dtype=np.int32)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    if a.ndim != 2:
        raise ValueError("curve must have shape (n, D)")
    return a


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed with status {rc}")


def dfd(p, q, metric=EUCLIDEAN, method="table"):
    """Discrete Frechet distance of two float32 curves, computed in FP64.

    method: "recursive" (Algorithm 1), "table" (Algorithm 3) or "rolling"
    (Algorithm 3 with two live rows).
    """
    lib = _load()
    p = _curve_f32(p)
    q = _curve_f32(q)
    if p.shape[1] != q.shape[1]:
        raise ValueError("dimension mismatch")
    fn = {"recursive": lib.ffdo_recursive, "table": lib.ffdo_table,
          "rolling": lib.ffdo_rolling}[method]
    out = ctypes.c_double()
    _check(fn(_ptr(p, ctypes.c_float), p.shape[0], _ptr(q, ctypes.c_float), q.shape[0],
              p.shape[1], int(metric), ctypes.byref(out)), method)
    return out.value


def dfd_table_full(p, q, metric=EUCLIDEAN):
    """The whole table M (n x m, FP64) of Algorithm 3."""
    lib = _load()
    p = _curve_f32(p)
    q = _curve_f32(q)
    M = np.empty((p.shape[0], q.shape[0]), dtype=np.float64)
    _check(lib.ffdo_table_full(_ptr(p, ctypes.c_float), p.shape[0], _ptr(q, ctypes.c_float),
                               q.shape[0], p.shape[1], int(metric), _ptr(M, ctypes.c_double)),
           "table_full")
    return M


def rolling_state(p, rows, q, metric=EUCLIDEAN):
    """Live row of the rolling form after `rows` rows of p (Theorem 1's O(Q) state)."""
    lib = _load()
    p = _curve_f32(p)
    q = _curve_f32(q)
    row = np.empty(q.shape[0], dtype=np.float64)
    _check(lib.ffdo_rolling_state(_ptr(p, ctypes.c_float), rows, _ptr(q, ctypes.c_float),
                                  q.shape[0], p.shape[1], int(metric), _ptr(row, ctypes.c_double)),
           "rolling_state")
    return row


def rolling_resume(p, row0, q, row, metric=EUCLIDEAN):
    """Finish the rolling form from a saved live row after row0 rows."""
    lib = _load()
    p = _curve_f32(p)
    q = _curve_f32(q)
    row = np.ascontiguousarray(row, dtype=np.float64)
    out = ctypes.c_double()
    _check(lib.ffdo_rolling_resume(_ptr(p, ctypes.c_float), row0, p.shape[0],
                                   _ptr(q, ctypes.c_float), q.shape[0], p.shape[1], int(metric),
                                   _ptr(row, ctypes.c_double), ctypes.byref(out)),
           "rolling_resume")
    return out.value


def dfd_i32(p, q, metric=SQEUCLIDEAN):
    """Exact discrete Frechet distance of int32 curves (int64); metric 1, 2 or 3."""
    lib = _load()
    p = _curve_i32(p)
    q = _curve_i32(q)
    if p.shape[1] != q.shape[1]:
        raise ValueError("dimension mismatch")
    out = ctypes.c_int64()
    _check(lib.ffdo_i32(_ptr(p, ctypes.c_int32), p.shape[0], _ptr(q, ctypes.c_int32),
                        q.shape[0], p.shape[1], int(metric), ctypes.byref(out)), "i32")
    return int(out.value)


def dfd_f32_replica(p, q, metric=EUCLIDEAN):
    """Float32 replica: d2 = dx*dx then fmaf(dk, dk, d2) for k >= 1, float32
    recurrence, one correctly rounded sqrt at the end for Euclidean."""
    lib = _load()
    p = _curve_f32(p)
    q = _curve_f32(q)
    out = ctypes.c_float()
    _check(lib.ffdo_f32_replica(_ptr(p, ctypes.c_float), p.shape[0], _ptr(q, ctypes.c_float),
                                q.shape[0], p.shape[1], int(metric), ctypes.byref(out)),
           "f32_replica")
    return np.float32(out.value)


def dtw(p, q, metric=EUCLIDEAN):
    """DTW (Appendix B) of two float32 curves in FP64; EUCLIDEAN takes the
    square root in every cell."""
    lib = _load()
    p = _curve_f32(p)
    q = _curve_f32(q)
    if p.shape[1] != q.shape[1]:
        raise ValueError("dimension mismatch")
    out = ctypes.c_double()
    _check(lib.ffdo_dtw(_ptr(p, ctypes.c_float), p.shape[0], _ptr(q, ctypes.c_float), q.shape[0],
                        p.shape[1], int(metric), ctypes.byref(out)), "dtw")
    return out.value


def dtw_i32(p, q, metric=SQEUCLIDEAN):
    """Exact DTW of int32 curves (int64); metric 1, 2 or 3."""
    lib = _load()
    p = _curve_i32(p)
    q = _curve_i32(q)
    if p.shape[1] != q.shape[1]:
        raise ValueError("dimension mismatch")
    out = ctypes.c_int64()
    _check(lib.ffdo_dtw_i32(_ptr(p, ctypes.c_int32), p.shape[0], _ptr(q, ctypes.c_int32),
                            q.shape[0], p.shape[1], int(metric), ctypes.byref(out)), "dtw_i32")
    return int(out.value)


def dtw_f32_replica(p, q, metric=EUCLIDEAN):
    """Float32 DTW replica: cell d2 as in dfd_f32_replica, a correctly
    rounded float32 sqrt per cell for Euclidean, v = min(...) + d in float32."""
    lib = _load()
    p = _curve_f32(p)
    q = _curve_f32(q)
    out = ctypes.c_float()
    _check(lib.ffdo_dtw_f32_replica(_ptr(p, ctypes.c_float), p.shape[0], _ptr(q, ctypes.c_float),
                                    q.shape[0], p.shape[1], int(metric), ctypes.byref(out)),
           "dtw_f32_replica")
    return np.float32(out.value)


def lev(p, q):
    """Levenshtein distance (Appendix B) of two int32 symbol sequences of
    shape (n, D) (a symbol is equal to another when every coordinate is)."""
    lib = _load()
    p = _curve_i32(p)
    q = _curve_i32(q)
    if p.shape[1] != q.shape[1]:
        raise ValueError("dimension mismatch")
    out = ctypes.c_int64()
    _check(lib.ffdo_lev(_ptr(p, ctypes.c_int32), p.shape[0], _ptr(q, ctypes.c_int32), q.shape[0],
                        p.shape[1], ctypes.byref(out)), "lev")
    return int(out.value)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def dfd_pairs(P, p_start, p_len, Q, q_start, q_len, metric=EUCLIDEAN, nthreads=1, order=None,
              measure="dfd"):
    """Many float32 pairs on a thread pool; returns FP64 distances
    (measure "dfd" or "dtw")."""
    lib = _load()
    P = _curve_f32(P)
    Q = _curve_f32(Q)
    ps, pl, qs, ql = _i64(p_start), _i64(p_len), _i64(q_start), _i64(q_len)
    n = ps.shape[0]
    out = np.empty(n, dtype=np.float64)
    ordp = None
    if order is not None:
        order = _i64(order)
        ordp = _ptr(order, ctypes.c_int64)
    fn = lib.ffdo_dtw_pairs if measure == "dtw" else lib.ffdo_pairs
    _check(fn(_ptr(P, ctypes.c_float), _ptr(ps, ctypes.c_int64),
              _ptr(pl, ctypes.c_int64), _ptr(Q, ctypes.c_float),
              _ptr(qs, ctypes.c_int64), _ptr(ql, ctypes.c_int64), n, P.shape[1],
              int(metric), ordp, int(nthreads), _ptr(out, ctypes.c_double)), "pairs")
    return out


def dfd_pairs_i32(P, p_start, p_len, Q, q_start, q_len, nthreads=1, order=None, measure="dfd",
                  metric=SQEUCLIDEAN):
    """Many int32 pairs on a thread pool; returns exact int64 squared distances
    (measure "dfd" or "dtw")."""
    lib = _load()
    P = _curve_i32(P)
    Q = _curve_i32(Q)
    ps, pl, qs, ql = _i64(p_start), _i64(p_len), _i64(q_start), _i64(q_len)
    n = ps.shape[0]
    out = np.empty(n, dtype=np.int64)
    ordp = None
    if order is not None:
        order = _i64(order)
        ordp = _ptr(order, ctypes.c_int64)
    fn = lib.ffdo_dtw_pairs_i32 if measure == "dtw" else lib.ffdo_pairs_i32
    _check(fn(_ptr(P, ctypes.c_int32), _ptr(ps, ctypes.c_int64),
              _ptr(pl, ctypes.c_int64), _ptr(Q, ctypes.c_int32),
              _ptr(qs, ctypes.c_int64), _ptr(ql, ctypes.c_int64), n, P.shape[1],
              int(metric), ordp, int(nthreads), _ptr(out, ctypes.c_int64)), "pairs_i32")
    return out


def dfd_batch(P, p_off, Q, q_off, metric=EUCLIDEAN, nthreads=1, order=None):
    """Pair k = (P[p_off[k]:p_off[k+1]], Q[q_off[k]:q_off[k+1]])."""
    p_off = _i64(p_off)
    q_off = _i64(q_off)
    return dfd_pairs(P, p_off[:-1], np.diff(p_off), Q, q_off[:-1], np.diff(q_off), metric,
                     nthreads, order)


def dfd_batch_i32(P, p_off, Q, q_off, nthreads=1, order=None, metric=SQEUCLIDEAN):
    p_off = _i64(p_off)
    q_off = _i64(q_off)
    return dfd_pairs_i32(P, p_off[:-1], np.diff(p_off), Q, q_off[:-1], np.diff(q_off),
                         nthreads, order, metric=metric)


def _cross_index(q_off, db_off, rows=None):
    q_off = _i64(q_off)
    db_off = _i64(db_off)
    nq = q_off.shape[0] - 1
    ndb = db_off.shape[0] - 1
    qi = np.arange(nq, dtype=np.int64) if rows is None else _i64(rows)
    ii = np.repeat(qi, ndb)
    kk = np.tile(np.arange(ndb, dtype=np.int64), qi.shape[0])
    return (q_off[ii], q_off[ii + 1] - q_off[ii], db_off[kk], db_off[kk + 1] - db_off[kk],
            qi.shape[0], ndb)


def dfd_cross(Qs, q_off, DB, db_off, metric=EUCLIDEAN, nthreads=1, rows=None):
    """out[i, k] = delta(query i, database curve k); `rows` selects query rows."""
    ps, pl, qs, ql, nr, ndb = _cross_index(q_off, db_off, rows)
    return dfd_pairs(Qs, ps, pl, DB, qs, ql, metric, nthreads).reshape(nr, ndb)


def dfd_cross_i32(Qs, q_off, DB, db_off, nthreads=1, rows=None, metric=SQEUCLIDEAN):
    ps, pl, qs, ql, nr, ndb = _cross_index(q_off, db_off, rows)
    return dfd_pairs_i32(Qs, ps, pl, DB, qs, ql, nthreads, metric=metric).reshape(nr, ndb)


def dtw_batch(P, p_off, Q, q_off, metric=EUCLIDEAN, nthreads=1, order=None):
    p_off = _i64(p_off)
    q_off = _i64(q_off)
    return dfd_pairs(P, p_off[:-1], np.diff(p_off), Q, q_off[:-1], np.diff(q_off), metric,
                     nthreads, order, measure="dtw")


def dtw_batch_i32(P, p_off, Q, q_off, nthreads=1, order=None, metric=SQEUCLIDEAN):
    p_off = _i64(p_off)
    q_off = _i64(q_off)
    return dfd_pairs_i32(P, p_off[:-1], np.diff(p_off), Q, q_off[:-1], np.diff(q_off),
                         nthreads, order, measure="dtw", metric=metric)


def dtw_cross(Qs, q_off, DB, db_off, metric=EUCLIDEAN, nthreads=1, rows=None):
    ps, pl, qs, ql, nr, ndb = _cross_index(q_off, db_off, rows)
    return dfd_pairs(Qs, ps, pl, DB, qs, ql, metric, nthreads, measure="dtw").reshape(nr, ndb)


def dtw_cross_i32(Qs, q_off, DB, db_off, nthreads=1, rows=None, metric=SQEUCLIDEAN):
    ps, pl, qs, ql, nr, ndb = _cross_index(q_off, db_off, rows)
    return dfd_pairs_i32(Qs, ps, pl, DB, qs, ql, nthreads, measure="dtw", metric=metric).reshape(nr, ndb)


def lev_pairs(P, p_start, p_len, Q, q_start, q_len, nthreads=1, order=None):
    lib = _load()
    P = _curve_i32(P)
    Q = _curve_i32(Q)
    ps, pl, qs, ql = _i64(p_start), _i64(p_len), _i64(q_start), _i64(q_len)
    n = ps.shape[0]
    out = np.empty(n, dtype=np.int64)
    ordp = None
    if order is not None:
        order = _i64(order)
        ordp = _ptr(order, ctypes.c_int64)
    _check(lib.ffdo_lev_pairs(_ptr(P, ctypes.c_int32), _ptr(ps, ctypes.c_int64), _ptr(pl, ctypes.c_int64),
                              _ptr(Q, ctypes.c_int32), _ptr(qs, ctypes.c_int64), _ptr(ql, ctypes.c_int64), n,
                              P.shape[1], ordp, int(nthreads), _ptr(out, ctypes.c_int64)), "lev_pairs")
    return out


def lev_batch(P, p_off, Q, q_off, nthreads=1, order=None):
    p_off = _i64(p_off)
    q_off = _i64(q_off)
    return lev_pairs(P, p_off[:-1], np.diff(p_off), Q, q_off[:-1], np.diff(q_off), nthreads, order)


def lev_cross(Qs, q_off, DB, db_off, nthreads=1, rows=None):
    ps, pl, qs, ql, nr, ndb = _cross_index(q_off, db_off, rows)
    return lev_pairs(Qs, ps, pl, DB, qs, ql, nthreads).reshape(nr, ndb)


def decide(values, eps):
    """The decider's answer from distances: delta if delta <= eps, else +inf
    (the question "is delta <= eps?" with the distance kept when it is)."""
    v = np.asarray(values)
    return np.where(v <= eps, v, np.inf).astype(v.dtype)


def knn(values, k):
    """Indices and distances of the k smallest values, in increasing value,
    ties by the smaller index; past the end: index -1 and +inf."""
    v = np.asarray(values)
    order = np.lexsort((np.arange(len(v)), v))[:k]
    idx = np.full(k, -1, dtype=np.int64)
    dist = np.full(k, np.inf, dtype=v.dtype)
    idx[:len(order)] = order
    dist[:len(order)] = v[order]
    return idx, dist


def now():
    """Monotonic clock of the C library (seconds)."""
    return _load().ffdo_now()
