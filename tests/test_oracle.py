"""Pins for the CPU oracle (no GPU).

Each test ties the oracle to something other than itself: brute force over
all couplings, a hand-worked example, closed forms, or invariants that the
definition implies.  The last group plants mistakes in copies of the
recurrence and checks that the pins catch each of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute, paper_forms
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
METHODS = ("recursive", "table", "rolling")


def _rng(seed):
    return np.random.default_rng(seed)


def _tiny_cases(seed, count, maxlen=6):
    """Random tiny float32 curves: N(0,1) walks, a two-value alphabet (ties)
    and small integers, D in {1, 2, 3}."""
    rng = _rng(seed)
    out = []
    for c in range(count):
        n = int(rng.integers(1, maxlen + 1))
        m = int(rng.integers(1, maxlen + 1))
        D = int(rng.integers(1, 4))
        kind = c % 3
        if kind == 0:
            p = workloads.walk(rng, n, D)
            q = workloads.walk(rng, m, D)
        elif kind == 1:
            p = rng.integers(0, 2, size=(n, D)).astype(np.float32)
            q = rng.integers(0, 2, size=(m, D)).astype(np.float32)
        else:
            p = rng.integers(-3, 4, size=(n, D)).astype(np.float32)
            q = rng.integers(-3, 4, size=(m, D)).astype(np.float32)
        out.append((p, q))
    return out


# --------------------------------------------------------------- hand example

def test_hand_example():
    g = json.load(open(os.path.join(GOLDEN, "hand_example.json")))
    p = np.array(g["p"], dtype=np.float32)
    q = np.array(g["q"], dtype=np.float32)
    np.testing.assert_array_equal(brute.ground_matrix(p, q), np.array(g["d"]))
    np.testing.assert_array_equal(oracle.dfd_table_full(p, q), np.array(g["M"]))
    for method in METHODS:
        assert oracle.dfd(p, q, method=method) == g["delta"]
    assert brute.brute(p, q) == g["delta"]
    assert paper_forms.fast(g["d"]) == g["delta"]
    assert paper_forms.inplace(g["d"]) == g["delta"]
    assert paper_forms.linear(p, q, paper_forms.euclid_f64) == g["delta"]
    # the optimal coupling attains the value
    c = [(i - 1, j - 1) for i, j in g["optimal_coupling_1based"]]
    assert max(g["d"][i][j] for i, j in c) == g["delta"]


def test_linear_row_trace_matches_hand_example():
    """Algorithm 5's live row after each row i equals row i of M."""
    g = json.load(open(os.path.join(GOLDEN, "hand_example.json")))
    p = np.array(g["p"], dtype=np.float32)
    q = np.array(g["q"], dtype=np.float32)
    for i in range(1, p.shape[0] + 1):
        row = oracle.rolling_state(p, i, q)
        np.testing.assert_array_equal(row, np.array(g["linear_row_trace"][i - 1]))


# ---------------------------------------------------- coupling enumerator itself

@pytest.mark.parametrize("P,Q", [(1, 1), (1, 5), (2, 2), (3, 4), (5, 5), (7, 7)])
def test_coupling_count_is_delannoy(P, Q):
    cs = list(brute.couplings(P, Q))
    assert len(cs) == brute.delannoy(P - 1, Q - 1)
    assert len({tuple(c) for c in cs}) == len(cs)
    for c in cs:
        assert c[0] == (0, 0) and c[-1] == (P - 1, Q - 1)
        for (a, b), (x, y) in zip(c, c[1:]):
            assert (x - a, y - b) in ((1, 0), (0, 1), (1, 1))


# --------------------------------------------------- P1: brute force agreement

def test_all_methods_equal_brute_force():
    for p, q in _tiny_cases(11, 240):
        want = brute.brute(p, q)
        for method in METHODS:
            assert oracle.dfd(p, q, method=method) == want
        want_sq = brute.brute(p, q, squared=True)
        assert oracle.dfd(p, q, oracle.SQEUCLIDEAN, "table") == want_sq


def test_up_to_seven_points_brute_force():
    rng = _rng(12)
    for _ in range(12):
        p = workloads.walk(rng, 7, 2)
        q = workloads.walk(rng, 7, 2)
        assert oracle.dfd(p, q) == brute.brute(p, q)


def test_int_exact_equals_brute_force():
    rng = _rng(13)
    for _ in range(150):
        n, m, D = (int(rng.integers(1, 7)), int(rng.integers(1, 7)), int(rng.integers(1, 4)))
        p = rng.integers(-(1 << 15), 1 << 15, size=(n, D), dtype=np.int32)
        q = rng.integers(-(1 << 15), 1 << 15, size=(m, D), dtype=np.int32)
        assert oracle.dfd_i32(p, q) == brute.brute_int(p, q)


def test_int_extreme_values_exact():
    """Largest squared distance of the int workload, 2 * 65535^2 > 2^32."""
    lo, hi = -(1 << 15), (1 << 15) - 1
    p = np.array([[lo, lo], [hi, lo]], dtype=np.int32)
    q = np.array([[hi, hi]], dtype=np.int32)
    want = 2 * 65535 ** 2
    assert want > 2 ** 32
    assert oracle.dfd_i32(p, q) == want
    # float32 holds these integers exactly and FP64 squares them exactly
    assert oracle.dfd(p.astype(np.float32), q.astype(np.float32), oracle.SQEUCLIDEAN) == want


# ------------------------------------------------------------ P2: special cases

def test_single_point_curves_reduce_to_max():
    rng = _rng(14)
    for _ in range(40):
        m = int(rng.integers(1, 40))
        D = int(rng.integers(1, 4))
        p = workloads.walk(rng, 1, D)
        q = workloads.walk(rng, m, D)
        d = brute.ground_matrix(p, q)
        assert oracle.dfd(p, q) == d.max()
        assert oracle.dfd(q, p) == d.max()
    p = np.array([[3.0, 4.0]], dtype=np.float32)
    q = np.zeros((1, 2), dtype=np.float32)
    assert oracle.dfd(p, q) == 5.0


# ------------------------------------------------------- P3/P4: closed forms

def test_identical_curves_are_zero():
    rng = _rng(15)
    for n in (1, 2, 17, 300):
        p = workloads.walk(rng, n, 3)
        for method in METHODS:
            assert oracle.dfd(p, p, method=method) == 0.0


def test_translated_copy_is_the_translation_length():
    """delta(q + c, q) = ||c||: both end pairs give the lower bound and the
    diagonal coupling gives the upper bound.  Integer data keeps it exact."""
    rng = _rng(16)
    for _ in range(20):
        n = int(rng.integers(1, 200))
        q = workloads.paper_walk(rng, n, 2)
        c = rng.integers(-20, 21, size=2).astype(np.float32)
        p = q + c
        want = math.sqrt(float(c[0]) ** 2 + float(c[1]) ** 2)
        assert oracle.dfd(p, q) == want
        assert oracle.dfd(p, q, oracle.SQEUCLIDEAN) == float(c[0]) ** 2 + float(c[1]) ** 2


# ---------------------------------------------------- P5-P7: bounds

def _hausdorff(d):
    return max(d.min(axis=1).max(), d.min(axis=0).max())


def _diagonal_coupling(n, m):
    steps = max(n, m)
    return [(round(k * (n - 1) / (steps - 1)) if steps > 1 else 0,
             round(k * (m - 1) / (steps - 1)) if steps > 1 else 0) for k in range(steps)]


def test_bounds_hold():
    rng = _rng(17)
    for _ in range(60):
        n, m = int(rng.integers(1, 120)), int(rng.integers(1, 120))
        p = workloads.walk(rng, n, 2)
        q = workloads.walk(rng, m, 2)
        d = brute.ground_matrix(p, q)
        delta = oracle.dfd(p, q)
        assert delta >= max(d[0, 0], d[-1, -1])           # P5: both end pairs
        assert delta >= _hausdorff(d)                      # P6: Frechet >= Hausdorff
        cpl = _diagonal_coupling(n, m)
        assert delta <= max(d[i, j] for i, j in cpl)       # P7: any coupling
        assert delta <= d.max()
        assert delta in set(d.ravel().tolist())            # the DP only selects


# ---------------------------------------------- P8-P10: exact invariances

def test_symmetry_reversal_and_repetition_are_bit_exact():
    rng = _rng(18)
    for _ in range(60):
        n, m, D = int(rng.integers(1, 90)), int(rng.integers(1, 90)), int(rng.integers(1, 4))
        p = workloads.walk(rng, n, D)
        q = workloads.walk(rng, m, D)
        delta = oracle.dfd(p, q)
        assert oracle.dfd(q, p) == delta
        assert oracle.dfd(p[::-1], q[::-1]) == delta
        # repeating points (Sec. 4 footnote), including padding with the last point
        reps = rng.integers(1, 4, size=n)
        assert oracle.dfd(np.repeat(p, reps, axis=0), q) == delta
        pad = np.concatenate([p, np.repeat(p[-1:], 7, axis=0)])
        assert oracle.dfd(pad, q) == delta
        padq = np.concatenate([np.repeat(q[:1], 3, axis=0), q])
        assert oracle.dfd(p, padq) == delta


def test_triangle_inequality():
    rng = _rng(19)
    for _ in range(40):
        a = workloads.walk(rng, int(rng.integers(1, 60)), 2)
        b = workloads.walk(rng, int(rng.integers(1, 60)), 2)
        c = workloads.walk(rng, int(rng.integers(1, 60)), 2)
        ab, bc, ac = oracle.dfd(a, b), oracle.dfd(b, c), oracle.dfd(a, c)
        assert ac <= ab + bc + 1e-12 * (ab + bc)


def test_squared_metric_is_square_of_euclidean():
    rng = _rng(20)
    for _ in range(40):
        p = workloads.walk(rng, int(rng.integers(1, 80)), 3)
        q = workloads.walk(rng, int(rng.integers(1, 80)), 3)
        e = oracle.dfd(p, q)
        s = oracle.dfd(p, q, oracle.SQEUCLIDEAN)
        assert math.sqrt(s) == e   # sqrt is monotone and correctly rounded


def test_power_of_two_scaling_is_exact():
    rng = _rng(21)
    for _ in range(30):
        p = workloads.walk(rng, int(rng.integers(1, 70)), 2)
        q = workloads.walk(rng, int(rng.integers(1, 70)), 2)
        for k in (-3, 5):
            s = np.float32(2.0 ** k)
            assert oracle.dfd(p * s, q * s) == oracle.dfd(p, q) * 2.0 ** k


# ------------------------------------------- P14: the paper's branch-free forms

def test_paper_forms_equal_oracle_bit_exact():
    for p, q in _tiny_cases(22, 150, maxlen=9):
        d = brute.ground_matrix(p, q)
        want = oracle.dfd(p, q)
        assert paper_forms.fast(d) == want
        assert paper_forms.inplace(d) == want
        assert paper_forms.linear(p, q, paper_forms.euclid_f64) == want
    rng = _rng(23)
    for _ in range(10):
        p = workloads.walk(rng, int(rng.integers(20, 60)), 2)
        q = workloads.walk(rng, int(rng.integers(20, 60)), 2)
        d = brute.ground_matrix(p, q)
        assert paper_forms.fast(d) == oracle.dfd(p, q)


def test_scan_and_fold_operators():
    """Appendix A: the scan prepends its initial value (N+1 outputs), the
    same-type scan seeds with the first element (N outputs)."""
    add = lambda a, b: a + b
    assert paper_forms.scan(add, 10, [1, 2, 3]) == [10, 11, 13, 16]
    assert paper_forms.scan1(max, [3, 1, 4, 1, 5]) == [3, 3, 4, 4, 5]
    assert paper_forms.fold(add, 10, [1, 2, 3]) == 16
    assert paper_forms.fold1(max, [3, 1, 4]) == 4


def test_sequential_reading_of_shift_min_is_wrong():
    """Reading the vector assignment as an ascending in-place loop gives a
    prefix minimum, e.g. [1,5,9] -> [1,1,1] instead of [1,1,5]; brute force
    rejects it on some inputs while the simultaneous reading always agrees."""
    wrong = 0
    for p, q in _tiny_cases(24, 300, maxlen=6):
        d = brute.ground_matrix(p, q)
        want = brute.brute(p, q)
        assert paper_forms.fast(d) == want
        if paper_forms.fast(d, sequential_shift=True) != want:
            wrong += 1
    assert wrong > 0


# --------------------------------------------- checkpoint of the live row

def test_rolling_state_checkpoint_and_resume():
    rng = _rng(25)
    for _ in range(10):
        n, m = int(rng.integers(2, 150)), int(rng.integers(1, 150))
        p = workloads.walk(rng, n, 2)
        q = workloads.walk(rng, m, 2)
        k = int(rng.integers(1, n))
        row = oracle.rolling_state(p, k, q)
        np.testing.assert_array_equal(row, oracle.dfd_table_full(p, q)[k - 1])
        assert oracle.rolling_resume(p, k, q, row) == oracle.dfd(p, q)


# ------------------------------------------------------------ float replica

def test_f32_replica_on_integer_walks_is_the_rounded_oracle():
    """Paper-style walks keep every float32 squared distance an exact integer
    below 2^24, so the float replica selects the same cell as the oracle."""
    rng = _rng(26)
    for _ in range(30):
        p = workloads.paper_walk(rng, int(rng.integers(1, 300)), 2)
        q = workloads.paper_walk(rng, int(rng.integers(1, 300)), 2)
        want = oracle.dfd(p, q)
        assert oracle.dfd_f32_replica(p, q) == np.float32(want)
        assert oracle.dfd_f32_replica(p, q, oracle.SQEUCLIDEAN) == np.float32(
            oracle.dfd(p, q, oracle.SQEUCLIDEAN))


def test_f32_replica_within_tolerance_of_oracle():
    rng = _rng(27)
    for _ in range(40):
        D = int(rng.integers(1, 4))
        p = workloads.walk(rng, int(rng.integers(1, 200)), D)
        q = workloads.walk(rng, int(rng.integers(1, 200)), D)
        want = oracle.dfd(p, q)
        got = float(oracle.dfd_f32_replica(p, q))
        assert abs(got - want) <= 2e-6 * want


# ---------------------------------------------------------- thread pool driver

def test_pairs_pool_matches_single_calls_in_any_order():
    P, p_off, Q, q_off = workloads.random_pairs(28, 40, 1, 60, dim=2)
    want = np.array([oracle.dfd(P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]])
                     for k in range(40)])
    got = oracle.dfd_batch(P, p_off, Q, q_off, nthreads=4)
    np.testing.assert_array_equal(got, want)
    order = np.argsort(-(np.diff(p_off) * np.diff(q_off)))
    np.testing.assert_array_equal(oracle.dfd_batch(P, p_off, Q, q_off, nthreads=3, order=order), want)


def test_int_pool_and_cross():
    Qs, q_off, DB, db_off = workloads.cross_int(seed=29, nq=5, ndb=7, length=11)
    got = oracle.dfd_cross_i32(Qs, q_off, DB, db_off, nthreads=4)
    for i in range(5):
        for k in range(7):
            assert got[i, k] == oracle.dfd_i32(Qs[q_off[i]:q_off[i + 1]], DB[db_off[k]:db_off[k + 1]])


def test_invalid_arguments_rejected():
    p = np.zeros((0, 2), dtype=np.float32)
    q = np.zeros((3, 2), dtype=np.float32)
    with pytest.raises(ValueError):
        oracle.dfd(p, q)
    with pytest.raises(ValueError):
        oracle.dfd(q, q, metric=7)


# ------------------------------------------------- planted mistakes are caught

def _mutant_table(d, mutation):
    """A copy of the recurrence with one planted mistake (CPU only)."""
    P, Q = d.shape
    M = np.zeros_like(d)
    for i in range(P):
        for j in range(Q):
            if i == 0 and j == 0:
                v = d[0, 0]
            elif j == 0:
                v = max(M[i - 1, 0], d[i, 0]) if mutation != "col_no_max" else d[i, 0]
            elif i == 0:
                v = max(M[0, j - 1], d[0, j])
            else:
                up, diag, left = M[i - 1, j], M[i - 1, j - 1], M[i, j - 1]
                if mutation == "drop_diag":
                    v = max(min(up, left), d[i, j])
                elif mutation == "drop_left":
                    v = max(min(up, diag), d[i, j])
                elif mutation == "min_for_max":
                    v = min(min(up, diag, left), d[i, j])
                elif mutation == "max3":
                    v = max(max(up, diag, left), d[i, j])
                elif mutation == "transposed_diag":
                    v = max(min(up, M[i - 1, j - 1] if i < 2 else M[i - 2, j - 1], left), d[i, j])
                else:
                    v = max(min(up, diag, left), d[i, j])
            M[i, j] = v
    return M[-1, -1]


@pytest.mark.parametrize("mutation", ["drop_diag", "drop_left", "min_for_max", "max3",
                                      "col_no_max", "transposed_diag"])
def test_pins_catch_planted_mistakes(mutation):
    caught = 0
    for p, q in _tiny_cases(30, 200, maxlen=6):
        d = brute.ground_matrix(p, q)
        if _mutant_table(d, mutation) != brute.brute(p, q):
            caught += 1
    assert caught > 0
    # and the unmutated copy passes the same pin everywhere
    for p, q in _tiny_cases(30, 60, maxlen=6):
        d = brute.ground_matrix(p, q)
        assert _mutant_table(d, None) == brute.brute(p, q)
