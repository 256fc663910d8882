"""Pins for the Manhattan and Chebyshev ground distances in the CPU oracle
(no GPU).

Sec. 3 states that the method assumes nothing about the ground distance, so
the same recurrences (Eq. (1) and the DTW algorithm of Appendix B) run on
d_ij = sum_k |p_ik - q_jk| (Manhattan) or max_k |p_ik - q_jk| (Chebyshev).
The oracle is tied to brute force over all couplings (bit-exact), to the
one-dimensional case where all four ground distances coincide, to the norm
inequalities Chebyshev <= Euclidean <= Manhattan <= sqrt(D) Euclidean, which
carry over to both measures cell by cell, and to exact integer results.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
import workloads

MET = (oracle.MANHATTAN, oracle.CHEBYSHEV)


def _tiny(seed, count, maxlen=6):
    rng = np.random.default_rng(seed)
    out = []
    for c in range(count):
        n, m, D = int(rng.integers(1, maxlen + 1)), int(rng.integers(1, maxlen + 1)), int(rng.integers(1, 5))
        if c % 2:
            p = rng.integers(-3, 4, size=(n, D)).astype(np.float32)
            q = rng.integers(-3, 4, size=(m, D)).astype(np.float32)
        else:
            p, q = workloads.walk(rng, n, D), workloads.walk(rng, m, D)
        out.append((p, q))
    return out


def test_brute_force_bit_exact_both_measures():
    for p, q in _tiny(90, 150):
        for metric in MET:
            assert oracle.dfd(p, q, metric, "table") == brute.brute(p, q, metric=metric)
            assert oracle.dfd(p, q, metric, "recursive") == brute.brute(p, q, metric=metric)
            assert oracle.dtw(p, q, metric) == brute.brute_dtw(p, q, metric=metric)


def test_int_exact_equals_brute_force():
    rng = np.random.default_rng(91)
    for _ in range(100):
        n, m, D = int(rng.integers(1, 7)), int(rng.integers(1, 7)), int(rng.integers(1, 5))
        p = rng.integers(-(1 << 15), 1 << 15, size=(n, D)).astype(np.int32)
        q = rng.integers(-(1 << 15), 1 << 15, size=(m, D)).astype(np.int32)
        for metric in MET:
            assert oracle.dfd_i32(p, q, metric) == brute.brute_int(p, q, metric=metric)
            assert oracle.dtw_i32(p, q, metric) == brute.brute_dtw_int(p, q, metric=metric)


def test_one_dimension_all_metrics_coincide():
    rng = np.random.default_rng(92)
    for _ in range(40):
        n, m = int(rng.integers(1, 80)), int(rng.integers(1, 80))
        p, q = workloads.walk(rng, n, 1), workloads.walk(rng, m, 1)
        e = oracle.dfd(p, q, oracle.EUCLIDEAN, "rolling")
        w = oracle.dtw(p, q, oracle.EUCLIDEAN)
        for metric in MET:
            assert oracle.dfd(p, q, metric, "rolling") == e
            assert oracle.dtw(p, q, metric) == w
            assert oracle.dfd_f32_replica(p, q, metric) == oracle.dfd_f32_replica(p, q, oracle.EUCLIDEAN)


def test_norm_inequalities_carry_over():
    rng = np.random.default_rng(93)
    eps = 1e-12
    for _ in range(60):
        n, m, D = int(rng.integers(1, 60)), int(rng.integers(1, 60)), int(rng.integers(1, 5))
        p, q = workloads.walk(rng, n, D), workloads.walk(rng, m, D)
        for fn in (lambda mt: oracle.dfd(p, q, mt, "rolling"), lambda mt: oracle.dtw(p, q, mt)):
            c, e, l1 = fn(oracle.CHEBYSHEV), fn(oracle.EUCLIDEAN), fn(oracle.MANHATTAN)
            assert c <= e * (1 + eps) and e <= l1 * (1 + eps)
            assert l1 <= np.sqrt(D) * e * (1 + eps) and e <= np.sqrt(D) * c * (1 + eps)


def test_hand_example():
    # p = (0,0), (3,4); q = (3,0): cells |.|_1 = 3 and 4, |.|_inf = 3 and 4
    p = np.array([[0, 0], [3, 4]], dtype=np.float32)
    q = np.array([[3, 0]], dtype=np.float32)
    assert oracle.dfd(p, q, oracle.MANHATTAN) == 4.0 and oracle.dtw(p, q, oracle.MANHATTAN) == 7.0
    assert oracle.dfd(p, q, oracle.CHEBYSHEV) == 4.0 and oracle.dtw(p, q, oracle.CHEBYSHEV) == 7.0
    # p = (0,0), (1,1); q = (2,0): |.|_1 = 2, 2; |.|_inf = 2, 1
    p = np.array([[0, 0], [1, 1]], dtype=np.float32)
    q = np.array([[2, 0]], dtype=np.float32)
    assert oracle.dfd(p, q, oracle.MANHATTAN) == 2.0 and oracle.dtw(p, q, oracle.MANHATTAN) == 4.0
    assert oracle.dfd(p, q, oracle.CHEBYSHEV) == 2.0 and oracle.dtw(p, q, oracle.CHEBYSHEV) == 3.0


def test_f32_replica_within_bounds_and_exact_on_integers():
    rng = np.random.default_rng(94)
    for _ in range(30):
        n, m, D = int(rng.integers(1, 200)), int(rng.integers(1, 200)), int(rng.integers(1, 5))
        p, q = workloads.walk(rng, n, D), workloads.walk(rng, m, D)
        for metric in MET:
            want = oracle.dfd(p, q, metric, "rolling")
            assert abs(float(oracle.dfd_f32_replica(p, q, metric)) - want) <= 2e-6 * want
            w = oracle.dtw(p, q, metric)
            assert abs(float(oracle.dtw_f32_replica(p, q, metric)) - w) <= (n + m + 2 * D + 2) * 2.0 ** -24 * w
        pi = rng.integers(-50, 51, size=(n, D)).astype(np.float32)
        qi = rng.integers(-50, 51, size=(m, D)).astype(np.float32)
        for metric in MET:
            assert float(oracle.dfd_f32_replica(pi, qi, metric)) == oracle.dfd(pi, qi, metric, "rolling")
            assert float(oracle.dtw_f32_replica(pi, qi, metric)) == oracle.dtw(pi, qi, metric)


def test_pools_match_single_calls():
    P, p_off, Q, q_off = workloads.random_pairs(95, 30, 1, 100, dim=3)
    for metric in MET:
        got = oracle.dfd_batch(P, p_off, Q, q_off, metric=metric, nthreads=3)
        gw = oracle.dtw_batch(P, p_off, Q, q_off, metric=metric, nthreads=3)
        for k in range(len(p_off) - 1):
            p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
            assert got[k] == oracle.dfd(p, q, metric, "rolling")
            assert gw[k] == oracle.dtw(p, q, metric)
    Qi, qoi, Di, doi = workloads.cross_int(seed=96, nq=3, ndb=5, length=20, dim=3)
    for metric in MET:
        cr = oracle.dfd_cross_i32(Qi, qoi, Di, doi, nthreads=2, metric=metric)
        cw = oracle.dtw_cross_i32(Qi, qoi, Di, doi, nthreads=2, metric=metric)
        for i in range(3):
            for k in range(5):
                a, b = Qi[qoi[i]:qoi[i + 1]], Di[doi[k]:doi[k + 1]]
                assert cr[i, k] == oracle.dfd_i32(a, b, metric)
                assert cw[i, k] == oracle.dtw_i32(a, b, metric)


@pytest.mark.parametrize("mistake", ["no_abs", "sum_for_max"])
def test_pins_catch_a_wrong_cell_distance(mistake):
    """A copy of the recurrence fed a wrong cell distance fails the brute-force pin."""
    caught = 0
    for p, q in _tiny(97, 120):
        P = p.astype(np.float64)[:, None, :]
        Q = q.astype(np.float64)[None, :, :]
        if mistake == "no_abs":
            d = (P - Q).sum(axis=2)
            metric = oracle.MANHATTAN
        else:
            d = np.abs(P - Q).sum(axis=2)
            metric = oracle.CHEBYSHEV
        if brute.brute_from_matrix(d.tolist()) != brute.brute(p, q, metric=metric):
            caught += 1
    assert caught > 0
