"""The early-abandoning rule of the decider and the k-nearest search,
checked on full oracle tables (CPU, no GPU).

Eq. (1) makes M_ij the smallest, over monotone paths from (0, 0) to (i, j),
of the largest cell on the path, so delta = M_PQ is at least the smallest M
over any set of cells that every full path crosses.  The sweep tests, after
each group of 16 steps while lane 0 is inside the column curve, the set made
of every lane's current cells (rows of lane l at column t - l), the cell
just above each lane's top row at that column, the band above's bottom row
to the right of lane 0's column and, when bands follow, this band's bottom
row up to lane 63's column (a path may leave the band downwards there).
Here that set is taken from the FP64 table of the row curve padded to whole
bands (repeating its last point, which leaves delta unchanged) and must
never exceed delta; dropping any of its parts breaks the rule, which the
test also shows.
"""
import numpy as np
import pytest

import oracle
import workloads


def front_minima(M, R, m, parts=("cells", "above", "band", "bottom")):
    """Smallest value of the tested set at every check, band by band."""
    BR = 64 * R
    nb = M.shape[0] // BR
    out = []
    for b in range(nb):
        top = b * BR
        for t0 in range(0, m, 16):
            t = t0 + 15
            if t > m - 1:
                break
            vals = [np.inf]
            for lane in range(64):
                c = t - lane
                if c < 0:
                    break
                if "cells" in parts:
                    vals.extend(M[top + lane * R: top + lane * R + R, c])
                if "above" in parts and (lane > 0 or b > 0):
                    vals.append(M[top + lane * R - 1, c])
            if "band" in parts and b > 0 and t + 1 < m:
                vals.append(M[top - 1, t + 1:].min())
            if "bottom" in parts and b < nb - 1 and t - 63 >= 0:
                vals.append(M[top + BR - 1, :t - 63 + 1].min())
            out.append(min(vals))
    return out


def padded_table(p, q, R):
    BR = 64 * R
    n = p.shape[0]
    rows = -(-n // BR) * BR
    pe = np.concatenate([p, np.repeat(p[-1:], rows - n, axis=0)])
    return oracle.dfd_table_full(pe, q, oracle.SQEUCLIDEAN)


@pytest.mark.parametrize("R", [1, 2])
def test_front_never_exceeds_delta(R):
    rng = np.random.default_rng(800 + R)
    checks = 0
    for _ in range(25):
        n, m = int(rng.integers(1, 320)), int(rng.integers(1, 140))
        p, q = workloads.walk(rng, n, 2), workloads.walk(rng, m, 2)
        M = padded_table(p, q, R)
        delta = oracle.dfd(p, q, oracle.SQEUCLIDEAN, "table")
        assert M[n - 1, m - 1] == delta and M[-1, m - 1] == delta
        for f in front_minima(M, R, m):
            assert f <= delta
            checks += 1
    assert checks > 100


def test_incomplete_sets_break_the_rule():
    """Without the cells above each lane, the band above's row or this
    band's bottom row, the tested set can exceed delta (the sweep would
    drop a pair whose distance is below the threshold)."""
    rng = np.random.default_rng(810)
    broken = {"no_above": 0, "no_band": 0, "no_bottom": 0}
    for _ in range(60):
        n, m = int(rng.integers(65, 200)), int(rng.integers(40, 120))
        p = workloads.walk(rng, n, 2)
        q = (p[np.linspace(0, n - 1, m).astype(int)] + 0.05 * rng.standard_normal((m, 2))).astype(np.float32)
        M = padded_table(p, q, 1)
        delta = oracle.dfd(p, q, oracle.SQEUCLIDEAN, "table")
        broken["no_above"] += any(f > delta for f in front_minima(M, 1, m, ("cells", "band", "bottom")))
        broken["no_band"] += any(f > delta for f in front_minima(M, 1, m, ("cells", "above", "bottom")))
        broken["no_bottom"] += any(f > delta for f in front_minima(M, 1, m, ("cells", "above", "band")))
    assert min(broken.values()) > 0, broken


def test_decide_and_knn_helpers():
    v = np.array([3.0, 1.0, 2.0, 1.0, np.inf], dtype=np.float32)
    np.testing.assert_array_equal(oracle.decide(v, 2.0), [np.inf, 1.0, 2.0, 1.0, np.inf])
    idx, dist = oracle.knn(v, 3)
    assert idx.tolist() == [1, 3, 2] and dist.tolist() == [1.0, 1.0, 2.0]
    idx, dist = oracle.knn(v[:2], 4)
    assert idx.tolist() == [1, 0, -1, -1] and np.isinf(dist[2:]).all()
    # against a plain selection loop
    rng = np.random.default_rng(811)
    w = rng.integers(0, 20, size=200).astype(np.float32)
    idx, dist = oracle.knn(w, 17)
    rest = list(range(200))
    for i in range(17):
        best = min(rest, key=lambda j: (w[j], j))
        rest.remove(best)
        assert idx[i] == best and dist[i] == w[best]
