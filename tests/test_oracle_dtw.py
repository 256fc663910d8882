"""Pins for the DTW part of the CPU oracle (Appendix B; no GPU).

Each test ties ``oracle.dtw*`` to something other than itself: hand-worked
tables, brute force over all couplings, the paper's own scan/fold form,
closed forms for single-point curves, and bounds that follow from the
definitions (a coupling's sum is at least its largest term and at most
n + m - 1 times it).  The last group plants mistakes in copies of the
recurrence and checks that the pins catch each of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute, paper_forms
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U32 = 2.0 ** -24


def _tiny_cases(seed, count, maxlen=6):
    """Random tiny float32 curves (walks, a two-value alphabet with ties,
    small integers), D in {1, 2, 3}."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(count):
        n = int(rng.integers(1, maxlen + 1))
        m = int(rng.integers(1, maxlen + 1))
        D = int(rng.integers(1, 4))
        kind = c % 3
        if kind == 0:
            p, q = workloads.walk(rng, n, D), workloads.walk(rng, m, D)
        elif kind == 1:
            p = rng.integers(0, 2, size=(n, D)).astype(np.float32)
            q = rng.integers(0, 2, size=(m, D)).astype(np.float32)
        else:
            p = rng.integers(-3, 4, size=(n, D)).astype(np.float32)
            q = rng.integers(-3, 4, size=(m, D)).astype(np.float32)
        out.append((p, q))
    return out


def test_dtw_hand_examples():
    g = json.load(open(os.path.join(GOLDEN, "dtw_hand_example.json")))
    for c in g["cases"]:
        metric = oracle.SQEUCLIDEAN if c["metric"] == "sqeuclidean" else oracle.EUCLIDEAN
        p = np.array(c["p"], dtype=np.float32)
        q = np.array(c["q"], dtype=np.float32)
        d = brute.ground_matrix(p, q, squared=metric == oracle.SQEUCLIDEAN)
        np.testing.assert_array_equal(d, np.array(c["d"]))
        np.testing.assert_array_equal(np.array(paper_forms.dtw_rows(d)), np.array(c["M"]))
        assert oracle.dtw(p, q, metric) == c["dtw"]
        assert oracle.dtw_f32_replica(p, q, metric) == np.float32(c["dtw"])
        assert oracle.dfd(p, q, metric) == c["dfd"]
        assert oracle.dtw_i32(p.astype(np.int32), q.astype(np.int32)) == (
            c["dtw"] if metric == oracle.SQEUCLIDEAN else oracle.dtw_i32(p.astype(np.int32), q.astype(np.int32)))


def test_dtw_equals_brute_force_bit_exact():
    """Rounding is monotone, so the recurrence's value is the smallest
    path-order sum over all couplings, bit for bit."""
    for p, q in _tiny_cases(70, 150):
        for metric in (oracle.EUCLIDEAN, oracle.SQEUCLIDEAN):
            want = brute.brute_dtw(p, q, squared=metric == oracle.SQEUCLIDEAN)
            assert oracle.dtw(p, q, metric) == want


def test_dtw_int_exact_equals_brute_force():
    rng = np.random.default_rng(71)
    for _ in range(120):
        n, m, D = (int(v) for v in (rng.integers(1, 7), rng.integers(1, 7), rng.integers(1, 4)))
        p = rng.integers(-(1 << 15), 1 << 15, size=(n, D)).astype(np.int32)
        q = rng.integers(-(1 << 15), 1 << 15, size=(m, D)).astype(np.int32)
        assert oracle.dtw_i32(p, q) == brute.brute_dtw_int(p, q)


def test_dtw_paper_form_bit_exact():
    """Algorithm B.1 (scan/fold, last element of the final row) equals the
    oracle bit for bit on inputs beyond brute-force size."""
    rng = np.random.default_rng(72)
    for _ in range(30):
        n, m, D = (int(v) for v in (rng.integers(1, 40), rng.integers(1, 40), rng.integers(1, 4)))
        p, q = workloads.walk(rng, n, D), workloads.walk(rng, m, D)
        for metric in (oracle.EUCLIDEAN, oracle.SQEUCLIDEAN):
            d = brute.ground_matrix(p, q, squared=metric == oracle.SQEUCLIDEAN)
            assert paper_forms.dtw(d) == oracle.dtw(p, q, metric)


def test_dtw_sequential_reading_of_shift_min_is_wrong():
    """The shifted minimum read as an in-place ascending loop gives other
    values (a prefix minimum), so the simultaneous reading is the one that
    matches the definition."""
    differ = 0
    for p, q in _tiny_cases(73, 80):
        d = brute.ground_matrix(p, q)
        if paper_forms.dtw(d, sequential_shift=True) != brute.brute_dtw(p, q):
            differ += 1
    assert differ > 0


def test_dtw_single_point_curves_are_sums():
    rng = np.random.default_rng(74)
    for _ in range(40):
        m, D = int(rng.integers(1, 50)), int(rng.integers(1, 4))
        p = workloads.walk(rng, 1, D)
        q = workloads.walk(rng, m, D)
        for metric in (oracle.EUCLIDEAN, oracle.SQEUCLIDEAN):
            row = brute.ground_matrix(p, q, squared=metric == oracle.SQEUCLIDEAN)[0]
            total = row[0]
            for v in row[1:]:
                total = total + v
            assert oracle.dtw(p, q, metric) == total
            assert oracle.dtw(q, p, metric) == total


def test_dtw_identity_symmetry_and_translation_bound():
    rng = np.random.default_rng(75)
    for _ in range(40):
        n, m, D = (int(v) for v in (rng.integers(1, 60), rng.integers(1, 60), rng.integers(1, 4)))
        p, q = workloads.walk(rng, n, D), workloads.walk(rng, m, D)
        assert oracle.dtw(p, p) == 0.0
        for metric in (oracle.EUCLIDEAN, oracle.SQEUCLIDEAN):
            # the transposed table runs the same operations on the same values
            assert oracle.dtw(p, q, metric) == oracle.dtw(q, p, metric)
            assert oracle.dtw_f32_replica(p, q, metric) == oracle.dtw_f32_replica(q, p, metric)
        # a translated copy: the diagonal coupling pays ||c|| in each of its
        # n cells, so DTW is at most n ||c|| (other couplings may pay less)
        c = np.float32(0.5)
        assert oracle.dtw(p, p + c) <= n * np.sqrt(D) * 0.5 * (1 + 1e-6)  # p + c is rounded to float32


def test_dtw_bounds_against_frechet():
    """DFD <= DTW <= (n + m - 1) DFD, and DTW >= max(n, m) min_ij d_ij."""
    rng = np.random.default_rng(76)
    for _ in range(60):
        n, m, D = (int(v) for v in (rng.integers(1, 50), rng.integers(1, 50), rng.integers(1, 4)))
        p, q = workloads.walk(rng, n, D), workloads.walk(rng, m, D)
        for metric in (oracle.EUCLIDEAN, oracle.SQEUCLIDEAN):
            w = oracle.dtw(p, q, metric)
            f = oracle.dfd(p, q, metric)
            dmin = brute.ground_matrix(p, q, squared=metric == oracle.SQEUCLIDEAN).min()
            assert f * (1 - 1e-12) <= w <= (n + m - 1) * f * (1 + 1e-12)
            assert w >= max(n, m) * dmin * (1 - 1e-12)


def test_dtw_f32_replica_within_summation_bound():
    """float32 DTW: each cell carries at most (D + 2) u of relative error
    (the fma chain and, for Euclidean, the square root), each of the at most
    n + m - 2 additions along the chosen coupling one more u; the minimum of
    values each within that bound of their exact counterparts is within it
    of the exact minimum."""
    rng = np.random.default_rng(77)
    for _ in range(40):
        n, m, D = (int(v) for v in (rng.integers(1, 300), rng.integers(1, 300), rng.integers(1, 5)))
        p, q = workloads.walk(rng, n, D), workloads.walk(rng, m, D)
        for metric in (oracle.EUCLIDEAN, oracle.SQEUCLIDEAN):
            want = oracle.dtw(p, q, metric)
            got = float(oracle.dtw_f32_replica(p, q, metric))
            tol = (n + m + D + 2) * U32 * 1.01
            assert abs(got - want) <= tol * want


def test_dtw_f32_replica_exact_on_small_integers():
    """Squared distances of small integer points and their sums stay below
    2^24, where float32 is exact: the replica equals the FP64 oracle."""
    rng = np.random.default_rng(78)
    for _ in range(40):
        n, m, D = (int(v) for v in (rng.integers(1, 200), rng.integers(1, 200), rng.integers(1, 4)))
        p = rng.integers(-20, 21, size=(n, D)).astype(np.float32)
        q = rng.integers(-20, 21, size=(m, D)).astype(np.float32)
        assert float(oracle.dtw_f32_replica(p, q, oracle.SQEUCLIDEAN)) == oracle.dtw(p, q, oracle.SQEUCLIDEAN)


def test_dtw_pools_match_single_calls():
    P, p_off, Q, q_off = workloads.random_pairs(79, 40, 1, 120, dim=2)
    got = oracle.dtw_batch(P, p_off, Q, q_off, nthreads=4)
    for k in range(len(p_off) - 1):
        assert got[k] == oracle.dtw(P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]])
    Qi, qoi, Di, doi = workloads.cross_int(seed=80, nq=3, ndb=7, length=30)
    cr = oracle.dtw_cross_i32(Qi, qoi, Di, doi, nthreads=3)
    for i in range(3):
        for k in range(7):
            assert cr[i, k] == oracle.dtw_i32(Qi[qoi[i]:qoi[i + 1]], Di[doi[k]:doi[k + 1]])
    bi = oracle.dtw_batch_i32(Qi, qoi, Di, doi[:4], nthreads=2)
    for k in range(3):
        assert bi[k] == oracle.dtw_i32(Qi[qoi[k]:qoi[k + 1]], Di[doi[k]:doi[k + 1]])


# ------------------------------------------------- planted mistakes are caught

def _mutant_dtw(d, mutation):
    """A copy of the DTW recurrence with one planted mistake (CPU only)."""
    P, Q = d.shape
    M = np.zeros_like(d)
    for i in range(P):
        for j in range(Q):
            if i == 0 and j == 0:
                v = d[0, 0]
            elif j == 0:
                v = M[i - 1, 0] + d[i, 0] if mutation != "col_no_sum" else d[i, 0]
            elif i == 0:
                v = M[0, j - 1] + d[0, j] if mutation != "row_max" else max(M[0, j - 1], d[0, j])
            else:
                up, diag, left = M[i - 1, j], M[i - 1, j - 1], M[i, j - 1]
                if mutation == "drop_diag":
                    v = min(up, left) + d[i, j]
                elif mutation == "drop_left":
                    v = min(up, diag) + d[i, j]
                elif mutation == "max_for_sum":
                    v = max(min(up, diag, left), d[i, j])
                elif mutation == "max3":
                    v = max(up, diag, left) + d[i, j]
                else:
                    v = min(up, diag, left) + d[i, j]
            M[i, j] = v
    return M[-1, -1]


@pytest.mark.parametrize("mutation", ["drop_diag", "drop_left", "max_for_sum", "max3", "col_no_sum",
                                      "row_max"])
def test_dtw_pins_catch_planted_mistakes(mutation):
    caught = 0
    for p, q in _tiny_cases(81, 200):
        d = brute.ground_matrix(p, q)
        if _mutant_dtw(d, mutation) != brute.brute_dtw(p, q):
            caught += 1
    assert caught > 0
    for p, q in _tiny_cases(81, 60):
        d = brute.ground_matrix(p, q)
        assert _mutant_dtw(d, None) == brute.brute_dtw(p, q)
