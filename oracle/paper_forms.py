"""The paper's branch-free formulations in FP64 (test infrastructure only).

Written from the descriptions in Sec. 3 and Appendix A of Meinert,
"Walking Your Frog Fast in 4 LoC" (arXiv 2404.05708):

* ``scan`` / ``fold``: the scan operator (Appendix A, Algorithm "scan") returns
  the initial value followed by every intermediate state, N + 1 values for N
  inputs; the fold operator (Appendix A, Algorithm "fold") returns only the
  final state.  When the state and the inputs have the same type, the first
  input is the initial value.
* ``fast``: Algorithm 2 (Theorem 1).  Row 1 of M is the running maximum of
  d_1; every later row applies ``next``: the element-wise shifted minimum of
  the previous row, then a scan of ``maxmin(a, x) = max(min(a, x1), x2)``
  seeded with max(a_1, x_1).  The answer is the last element.
* ``inplace``: Algorithm 4, which overwrites d: running maxima of the first
  column and row, then Eq. (1) over the interior.
* ``linear``: Algorithm 5, one row v of length Q.
* ``dtw``: the DTW algorithm of Appendix B (Algorithm B.1).  The first row is
  the +-scan of d_1; ``dtw_next`` applies the same shifted minimum and then
  a scan of ``dtw_min(a, x) = min(a, x1) + x2`` seeded with a_1 + x_1.  The
  printed return line lacks the closing "last element" bracket that
  Algorithm 2 has; it is read as the last element of the final row.
* ``levenshtein``: Algorithm B.2 (edit distance of symbol sequences), with
  its index vectors read 0-based.

The vector assignment "a_{2..Q} <- min(a_{1..Q-1}, a_{2..Q})" is read as a
simultaneous assignment (right-hand side evaluated before any element is
written).  ``sequential_shift=True`` switches to the other reading (an
ascending in-place loop, which turns the shifted minimum into a prefix
minimum); it exists so that tests can show this reading is wrong.
"""
import numpy as np


def scan(f, t0, xs):
    out = [t0]
    t = t0
    for x in xs:
        t = f(t, x)
        out.append(t)
    return out


def scan1(f, xs):
    """Same-type scan: the first element is the initial value (N outputs)."""
    return scan(f, xs[0], xs[1:])


def fold(f, t0, xs):
    t = t0
    for x in xs:
        t = f(t, x)
    return t


def fold1(f, xs):
    return fold(f, xs[0], xs[1:])


def _shift_min(a, sequential):
    a = list(a)
    if sequential:
        for j in range(1, len(a)):
            a[j] = min(a[j - 1], a[j])
        return a
    return [a[0]] + [min(a[j - 1], a[j]) for j in range(1, len(a))]


def maxmin(a, x):
    return max(min(a, x[0]), x[1])


def fast(d, sequential_shift=False):
    """Algorithm 2 on a distance matrix d (P x Q, any ordered numbers)."""
    d = [list(map(float, row)) for row in np.asarray(d).tolist()] if hasattr(d, "tolist") else d

    def nxt(a, x):
        a = _shift_min(a, sequential_shift)
        pairs = list(zip(a[1:], x[1:]))
        return scan(maxmin, max(a[0], x[0]), pairs)

    first = scan1(max, d[0])
    return fold(nxt, first, d[1:])[-1]


def inplace(d):
    """Algorithm 4: overwrite d; returns d_PQ."""
    d = np.array(d, dtype=np.float64, copy=True)
    P, Q = d.shape
    d[:, 0] = scan1(max, list(d[:, 0]))
    d[0, :] = scan1(max, list(d[0, :]))
    for i in range(1, P):
        for j in range(1, Q):
            d[i, j] = max(min(d[i - 1, j], d[i - 1, j - 1], d[i, j - 1]), d[i, j])
    return float(d[P - 1, Q - 1])


def linear(p, q, f, sequential_shift=False):
    """Algorithm 5: one live row v of length Q; f is the ground distance."""
    P, Q = len(p), len(q)
    v = scan1(max, [f(p[0], q[j]) for j in range(Q)])
    for i in range(1, P):
        v = _shift_min(v, sequential_shift)
        v[0] = max(v[0], f(p[i], q[0]))
        for j in range(1, Q):
            v[j] = max(min(v[j - 1], v[j]), f(p[i], q[j]))
    return v[Q - 1]


def dtw_min(a, x):
    return min(a, x[0]) + x[1]


def dtw_rows(d, sequential_shift=False):
    """Every row of Algorithm B.1's iteration (a scan in place of the final
    fold): row i is M_i of the DTW table."""
    d = [list(map(float, row)) for row in np.asarray(d).tolist()] if hasattr(d, "tolist") else d

    def nxt(a, x):
        a = _shift_min(a, sequential_shift)
        pairs = list(zip(a[1:], x[1:]))
        return scan(dtw_min, a[0] + x[0], pairs)

    first = scan1(lambda s, x: s + x, d[0])
    return scan(nxt, first, d[1:])


def dtw(d, sequential_shift=False):
    """Algorithm B.1 on a distance matrix d (P x Q): the last element of the
    final row."""
    return dtw_rows(d, sequential_shift)[-1][-1]


def levenshtein(d, one_based=False):
    """Algorithm B.2 on the matrix d_ij = [p_i != q_j] (P x Q).

    levenshtein_min(a, x) = min(a + 1, x); the first row is the same-type
    scan of levenshtein_min over iota_{1..Q} + d_1; every later row i applies
    the shifted update a_{2..Q} <- min(a_{1..Q-1} + x_{2..Q}, a_{2..Q} + 1)
    (simultaneous) and a scan seeded with min(iota_i + x_1, a_1 + 1).  The
    index vectors are read 0-based (iota_{1..Q} = 0 .. Q-1 for the first
    row, iota_{2..P} = 1 .. P-1 for the later ones); one_based=True takes
    the other reading, which tests show to be wrong."""
    d = [list(map(int, row)) for row in np.asarray(d).tolist()]
    P, Q = len(d), len(d[0])
    off = 1 if one_based else 0
    iota_q = [j + off for j in range(Q)]
    iota_p = [i + off for i in range(1, P)]

    def lmin(a, x):
        return min(a + 1, x)

    def nxt(a, ix):
        i, x = ix
        b = [a[0]] + [min(a[j - 1] + x[j], a[j] + 1) for j in range(1, len(a))]
        return scan(lmin, min(i + x[0], b[0] + 1), b[1:])

    first = scan1(lmin, [iota_q[j] + d[0][j] for j in range(Q)])
    return fold(nxt, first, list(zip(iota_p, d[1:])))[-1]


def euclid_f64(a, b):
    """||a - b|| in FP64, coordinates summed in order (the oracle's order)."""
    s = 0.0
    for x, y in zip(np.atleast_1d(a), np.atleast_1d(b)):
        t = float(x) - float(y)
        s = s + t * t
    return float(np.sqrt(s))

