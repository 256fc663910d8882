"""Brute force over all monotone couplings (test infrastructure only).

The discrete Frechet distance of Eiter and Mannila (cited in Sec. 2 of the
paper) is the minimum, over all couplings, of the largest ground distance
along the coupling.  A coupling of p (P points) and q (Q points) is a
sequence of index pairs that starts at (1, 1), ends at (P, Q) and advances by
(1, 0), (0, 1) or (1, 1) at every step.  This module enumerates every
coupling explicitly; it is exponential and meant for P, Q <= 7 (at most
Delannoy(6, 6) = 8989 couplings).

DTW (Appendix B) over the same couplings takes the sum of the ground
distances along a coupling instead of the largest one.
"""
import numpy as np


def ground_matrix(p, q, squared=False, metric=None):
    """d_ij = ||p_i - q_j|| in FP64 from the given coordinates (exact widening).

    The sum runs over coordinates in order, one term at a time, which is the
    same evaluation order as the C oracle.  metric (overrides `squared`):
    0 Euclidean, 1 squared Euclidean, 2 Manhattan, 3 Chebyshev.
    """
    if metric is None:
        metric = 1 if squared else 0
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if p.ndim == 1:
        p = p[:, None]
    if q.ndim == 1:
        q = q[:, None]
    s = np.zeros((p.shape[0], q.shape[0]), dtype=np.float64)
    for k in range(p.shape[1]):
        t = p[:, None, k] - q[None, :, k]
        if metric == 2:
            s = s + np.abs(t)
        elif metric == 3:
            s = np.maximum(s, np.abs(t))
        else:
            s = s + t * t
    return np.sqrt(s) if metric == 0 else s


def ground_matrix_int(p, q, metric=1):
    """Exact int64 distances of integer points: 1 squared Euclidean, 2
    Manhattan, 3 Chebyshev."""
    p = np.asarray(p, dtype=np.int64)
    q = np.asarray(q, dtype=np.int64)
    if p.ndim == 1:
        p = p[:, None]
    if q.ndim == 1:
        q = q[:, None]
    s = np.zeros((p.shape[0], q.shape[0]), dtype=np.int64)
    for k in range(p.shape[1]):
        t = p[:, None, k] - q[None, :, k]
        if metric == 2:
            s = s + np.abs(t)
        elif metric == 3:
            s = np.maximum(s, np.abs(t))
        else:
            s = s + t * t
    return s


def couplings(P, Q):
    """Yield every monotone coupling of index ranges [0, P) and [0, Q) (0-based)."""
    path = [(0, 0)]

    def walk(i, j):
        if i == P - 1 and j == Q - 1:
            yield list(path)
            return
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            a, b = i + di, j + dj
            if a < P and b < Q:
                path.append((a, b))
                yield from walk(a, b)
                path.pop()

    yield from walk(0, 0)


def brute_from_matrix(d):
    """min over couplings of max over the coupling of d (any ordered values)."""
    P, Q = len(d), len(d[0])
    best = None
    for c in couplings(P, Q):
        worst = max(d[i][j] for i, j in c)
        if best is None or worst < best:
            best = worst
    return best


def brute_dtw_from_matrix(d):
    """min over couplings of the sum along the coupling, added in path order
    (rounding is monotone, so this equals the table recurrence bit for bit)."""
    P, Q = len(d), len(d[0])
    best = None
    for c in couplings(P, Q):
        total = d[0][0]
        for i, j in c[1:]:
            total = total + d[i][j]
        if best is None or total < best:
            best = total
    return best


def brute_dtw(p, q, squared=False, metric=None):
    return float(brute_dtw_from_matrix(ground_matrix(p, q, squared, metric).tolist()))


def brute_dtw_int(p, q, metric=1):
    return int(brute_dtw_from_matrix(ground_matrix_int(p, q, metric).tolist()))


def brute(p, q, squared=False, metric=None):
    return float(brute_from_matrix(ground_matrix(p, q, squared, metric).tolist()))


def brute_int(p, q, metric=1):
    return int(brute_from_matrix(ground_matrix_int(p, q, metric).tolist()))


def delannoy(a, b):
    """Number of monotone couplings of lengths a+1 and b+1 (a check on `couplings`)."""
    from math import comb
    return sum(comb(a, k) * comb(b, k) * 2 ** k for k in range(min(a, b) + 1))
