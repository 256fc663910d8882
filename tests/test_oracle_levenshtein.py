"""Pins for the Levenshtein part of the CPU oracle (Appendix B, Algorithm
B.2; no GPU).

``oracle.lev`` is tied to hand-worked tables, to the recursive definition
on prefixes (a different formulation: the distance of the first i and j
symbols), to the paper's scan/fold algorithm with its index vectors read
0-based (the 1-based reading is shown to disagree), and to the properties
of an edit distance: symmetry, zero exactly on equal sequences, the bounds
|n - m| <= lev <= max(n, m), Hamming distance as an upper bound for equal
lengths, and the triangle inequality.  Planted mistakes are caught.
"""
import json
import os
from functools import lru_cache

import numpy as np
import pytest

import oracle
from oracle import paper_forms

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def seq(a, D=1):
    return np.asarray(a, dtype=np.int32).reshape(-1, D)


def recursive(p, q):
    """Distance of the prefixes of lengths i and j, by recursion on the last
    symbols (pure Python, small inputs)."""
    P = [tuple(r) for r in np.asarray(p).reshape(len(p), -1).tolist()]
    Q = [tuple(r) for r in np.asarray(q).reshape(len(q), -1).tolist()]

    @lru_cache(maxsize=None)
    def L(i, j):
        if i == 0:
            return j
        if j == 0:
            return i
        return min(L(i - 1, j) + 1, L(i, j - 1) + 1, L(i - 1, j - 1) + (P[i - 1] != Q[j - 1]))

    return L(len(P), len(Q))


def _cases(seed, count, maxlen=12, alphabet=3, D=1):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n, m = int(rng.integers(1, maxlen + 1)), int(rng.integers(1, maxlen + 1))
        out.append((rng.integers(0, alphabet, size=(n, D)).astype(np.int32),
                    rng.integers(0, alphabet, size=(m, D)).astype(np.int32)))
    return out


def test_hand_examples():
    g = json.load(open(os.path.join(GOLDEN, "levenshtein_hand_example.json")))
    for c in g["cases"]:
        p, q = seq(c["p"]), seq(c["q"])
        assert oracle.lev(p, q) == c["lev"]
        assert recursive(p, q) == c["lev"]
        # every cell of the table through the prefixes
        for i in range(len(c["p"])):
            for j in range(len(c["q"])):
                assert oracle.lev(p[:i + 1], q[:j + 1]) == c["M"][i][j]


def test_equals_recursive_definition():
    for p, q in _cases(120, 300) + _cases(121, 100, D=2, alphabet=2):
        assert oracle.lev(p, q) == recursive(p, q)


def match_form(p, q):
    """The cell form the kernels evaluate: on a symbol match the diagonal
    value, otherwise one more than the least of the three neighbours, with
    the boundary row j + 1 and column i + 1 (float32 integers, as on the
    device).  Equal to the recurrence because neighbouring values of the
    table differ by at most one."""
    P = [tuple(r) for r in np.asarray(p).reshape(len(p), -1).tolist()]
    Q = [tuple(r) for r in np.asarray(q).reshape(len(q), -1).tolist()]
    row = [np.float32(j + 1) for j in range(len(Q))]
    for i in range(len(P)):
        diag, left = np.float32(i), np.float32(i + 1)
        for j in range(len(Q)):
            v = diag if P[i] == Q[j] else min(row[j], left, diag) + np.float32(1)
            diag, left, row[j] = row[j], v, v
    return int(row[-1])


def test_kernel_match_form_equals_the_recurrence():
    cases = _cases(130, 400) + _cases(131, 150, D=2, alphabet=2) + _cases(132, 100, maxlen=30, alphabet=2)
    cases += [(seq([1] * 9), seq([1] * 5)), (seq([0, 1] * 6), seq([1, 0] * 6)), (seq([2]), seq([3] * 7))]
    for p, q in cases:
        assert match_form(p, q) == oracle.lev(p, q)


def test_paper_algorithm_zero_based_reading():
    differ = 0
    for p, q in _cases(122, 200, maxlen=9):
        d = (p[:, None, 0] != q[None, :, 0]).astype(int)
        assert paper_forms.levenshtein(d) == oracle.lev(p, q)
        differ += paper_forms.levenshtein(d, one_based=True) != oracle.lev(p, q)
    assert differ > 0


def test_metric_properties():
    rng = np.random.default_rng(123)
    for _ in range(150):
        n, m, k = (int(v) for v in rng.integers(1, 40, size=3))
        p, q, r = (rng.integers(0, 4, size=(L, 1)).astype(np.int32) for L in (n, m, k))
        a = oracle.lev(p, q)
        assert a == oracle.lev(q, p)
        assert abs(n - m) <= a <= max(n, m)
        assert oracle.lev(p, p) == 0
        assert (a == 0) == (n == m and np.array_equal(p, q))
        assert a <= oracle.lev(p, r) + oracle.lev(r, q)
        if n == m:
            assert a <= int(np.sum(p != q))


def test_pools_match_single_calls():
    rng = np.random.default_rng(124)
    curves = [rng.integers(0, 5, size=(int(L), 1)).astype(np.int32) for L in rng.integers(1, 60, size=24)]
    off = np.concatenate([[0], np.cumsum([len(c) for c in curves])]).astype(np.int64)
    X = np.concatenate(curves)
    got = oracle.lev_cross(X, off[:7], X, off, nthreads=4)
    for i in range(6):
        for k in range(24):
            assert got[i, k] == oracle.lev(curves[i], curves[k])
    pb = oracle.lev_pairs(X, off[:-1][:12], np.diff(off)[:12], X, off[:-1][12:], np.diff(off)[12:], nthreads=2)
    for k in range(12):
        assert pb[k] == oracle.lev(curves[k], curves[12 + k])


@pytest.mark.parametrize("mistake", ["no_diag_cost", "boundary_zero", "diag_plus_one"])
def test_pins_catch_planted_mistakes(mistake):
    def mutant(p, q):
        n, m = len(p), len(q)
        M = np.zeros((n + 1, m + 1), dtype=np.int64)
        M[0, :] = np.arange(m + 1) if mistake != "boundary_zero" else 0
        M[:, 0] = np.arange(n + 1) if mistake != "boundary_zero" else 0
        for i in range(1, n + 1):
            for j in range(1, m + 1):
                d = int(np.any(p[i - 1] != q[j - 1]))
                if mistake == "no_diag_cost":
                    d = 0
                elif mistake == "diag_plus_one":
                    d = d + 1
                M[i, j] = min(M[i - 1, j] + 1, M[i, j - 1] + 1, M[i - 1, j - 1] + d)
        return M[n, m]
    caught = sum(mutant(p, q) != recursive(p, q) for p, q in _cases(125, 80))
    assert caught > 0
