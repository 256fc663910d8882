"""GPU parity of dynamic time warping (Appendix B) through the C ABI.

Bars:
* squared Euclidean cells, float32: bit-identical to the float32 replica
  (the cell expression and the order of the additions along every coupling
  are fixed by the recurrence, minima are exact), and within a relative
  (n + m + D + 2) 2^-24 of the FP64 oracle;
* Euclidean cells, float32 (hardware square root, within 1 ulp): within a
  relative (n + m + D + 3) 2^-24 of the FP64 oracle;
* int32 coordinates: bit-exact against the int64 oracle;
* every launch shape, the batch, cross and single-pair forms, split bands
  and the Frechet calls on the same workspace give the same bits.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu):
    from paper_2404_05708_amd import ffd
    c = ffd.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def tol(n, m, D, metric):
    return (n + m + D + (3 if metric == oracle.EUCLIDEAN else 2)) * U32 * 1.01


def check_pair(got, p, q, metric):
    want = oracle.dtw(p, q, metric)
    n, D = p.shape
    m = q.shape[0]
    assert abs(float(got) - want) <= tol(n, m, D, metric) * want, (n, m, D, metric, float(got), want)
    if metric == oracle.SQEUCLIDEAN:
        assert np.float32(got) == oracle.dtw_f32_replica(p, q, metric), (n, m, D)


@pytest.mark.parametrize("R", [0, 1, 2, 4, 8])
def test_dtw_random_shapes_all_dims(ctx, R):
    rng = np.random.default_rng(200 + R)
    ctx.set_tuning(R, 0)
    try:
        for it in range(16):
            n = int(rng.integers(1, 700))
            m = int(rng.integers(1, 700))
            D = int(rng.integers(1, 5))
            p, q = workloads.walk(rng, n, D), workloads.walk(rng, m, D)
            for metric in (oracle.SQEUCLIDEAN, oracle.EUCLIDEAN):
                say(f"case: dtw pair R={R} n={n} m={m} D={D} metric={metric}")
                got = ctx.dtw_distance(dev(p), dev(q), metric=metric).item()
                check_pair(got, p, q, metric)
    finally:
        ctx.set_tuning(0, 0)


def test_dtw_edge_cases(ctx):
    rng = np.random.default_rng(210)
    cases = [(1, 1), (1, 300), (300, 1), (2, 2), (64, 64), (512, 80), (513, 79), (64 * 8, 64 * 8),
             (64 * 8 + 1, 17), (1000, 3000), (5000, 40)]
    for n, m in cases:
        p, q = workloads.walk(rng, n, 2), workloads.walk(rng, m, 2)
        for metric in (oracle.SQEUCLIDEAN, oracle.EUCLIDEAN):
            say(f"case: dtw edge n={n} m={m} metric={metric}")
            got = ctx.dtw_distance(dev(p), dev(q), metric=metric).item()
            assert ctx.last_errors() == 0
            check_pair(got, p, q, metric)
    # identical curves: every cell of the diagonal coupling is 0
    p = workloads.walk(rng, 777, 3)
    assert ctx.dtw_distance(dev(p), dev(p)).item() == 0.0


def test_dtw_batch_equals_pairs_cross_and_shapes(ctx):
    P, p_off, Q, q_off = workloads.random_pairs(211, 150, 1, 1500, dim=2)
    say("case: dtw batch of 150 pairs, squared")
    base = ctx.dtw_batch(dev(P), p_off, dev(Q), q_off, metric=oracle.SQEUCLIDEAN).cpu().numpy()
    want = oracle.dtw_batch(P, p_off, Q, q_off, metric=oracle.SQEUCLIDEAN, nthreads=8)
    for k in range(len(p_off) - 1):
        n, m = p_off[k + 1] - p_off[k], q_off[k + 1] - q_off[k]
        assert abs(base[k] - want[k]) <= tol(n, m, 2, oracle.SQEUCLIDEAN) * want[k]
    for k in range(0, len(p_off) - 1, 15):
        p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
        assert base[k] == oracle.dtw_f32_replica(p, q, oracle.SQEUCLIDEAN)
        assert ctx.dtw_distance(dev(p), dev(q), metric=oracle.SQEUCLIDEAN).item() == base[k]
    for R in (1, 2, 4, 8):
        for W in (1, 2):
            say(f"case: dtw batch, R={R} W={W}")
            ctx.set_tuning(R, W)
            try:
                got = ctx.dtw_batch(dev(P), p_off, dev(Q), q_off, metric=oracle.SQEUCLIDEAN).cpu().numpy()
            finally:
                ctx.set_tuning(0, 0)
            np.testing.assert_array_equal(got, base)
    say("case: dtw batch, every multi-band pair split over waves")
    ctx.set_tuning(2, 0)
    ctx.set_split(1e-9)
    try:
        got = ctx.dtw_batch(dev(P), p_off, dev(Q), q_off, metric=oracle.SQEUCLIDEAN).cpu().numpy()
        assert ctx.last_errors() == 0
    finally:
        ctx.set_split(0.0)
        ctx.set_tuning(0, 0)
    np.testing.assert_array_equal(got, base)
    say("case: dtw cross equals the batch of the same pairs")
    Qs, qo = workloads.concat([P[p_off[k]:p_off[k + 1]] for k in range(4)])
    DB, do = workloads.concat([Q[q_off[k]:q_off[k + 1]] for k in range(30)])
    cr = ctx.dtw_cross(dev(Qs), qo, dev(DB), do, metric=oracle.EUCLIDEAN).cpu().numpy()
    wcr = oracle.dtw_cross(Qs, qo, DB, do, metric=oracle.EUCLIDEAN, nthreads=8)
    for i in range(4):
        for k in range(30):
            n, m = qo[i + 1] - qo[i], do[k + 1] - do[k]
            assert abs(cr[i, k] - wcr[i, k]) <= tol(n, m, 2, oracle.EUCLIDEAN) * wcr[i, k]
            if k == i:
                pe = ctx.dtw_distance(dev(Qs[qo[i]:qo[i + 1]]), dev(DB[do[k]:do[k + 1]]),
                                      metric=oracle.EUCLIDEAN).item()
                assert pe == cr[i, k]


def test_dtw_and_frechet_share_a_workspace(ctx):
    """Plans differ per measure; alternating calls on one workspace must
    upload the right plan each time."""
    from paper_2404_05708_amd import ffd
    P, p_off, Q, q_off = workloads.random_pairs(212, 80, 1, 9000, dim=2)
    Pd, Qd = dev(P), dev(Q)
    ws = torch.empty(ctx.workspace_size(ffd.FFD_OP_BATCH, p_off, q_off, 2), dtype=torch.uint8, device="cuda:0")
    say("case: dtw / frechet alternating on one workspace, long curves")
    f1 = ctx.batch(Pd, p_off, Qd, q_off, workspace=ws).cpu().numpy()
    w1 = ctx.dtw_batch(Pd, p_off, Qd, q_off, metric=oracle.SQEUCLIDEAN, workspace=ws).cpu().numpy()
    f2 = ctx.batch(Pd, p_off, Qd, q_off, workspace=ws).cpu().numpy()
    w2 = ctx.dtw_batch(Pd, p_off, Qd, q_off, metric=oracle.SQEUCLIDEAN, workspace=ws).cpu().numpy()
    assert ctx.last_errors() == 0
    np.testing.assert_array_equal(f1, f2)
    np.testing.assert_array_equal(w1, w2)
    want = oracle.dtw_batch(P, p_off, Q, q_off, metric=oracle.SQEUCLIDEAN, nthreads=8)
    for k in range(len(p_off) - 1):
        n, m = p_off[k + 1] - p_off[k], q_off[k + 1] - q_off[k]
        assert abs(w1[k] - want[k]) <= tol(n, m, 2, oracle.SQEUCLIDEAN) * want[k]
    fw = oracle.dfd_batch(P, p_off, Q, q_off, nthreads=8)
    assert np.all(np.abs(f1 - fw) <= 2e-6 * fw)


def test_dtw_int_exact(ctx):
    Qi, qoi, Di, doi = workloads.cross_int(seed=213, nq=6, ndb=50, length=300)
    say("case: dtw int cross 6 x 50")
    got = ctx.dtw_cross_i32(dev(Qi), qoi, dev(Di), doi).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.dtw_cross_i32(Qi, qoi, Di, doi, nthreads=8))
    rng = np.random.default_rng(214)
    P, p_off, Q, q_off = workloads.random_pairs(215, 60, 1, 1300, dim=3)
    Pi = rng.integers(-(1 << 15), 1 << 15, size=P.shape).astype(np.int32)
    Qi2 = rng.integers(-(1 << 15), 1 << 15, size=Q.shape).astype(np.int32)
    say("case: dtw int batch 60 pairs, 3-D")
    got = ctx.dtw_batch_i32(dev(Pi), p_off, dev(Qi2), q_off).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.dtw_batch_i32(Pi, p_off, Qi2, q_off, nthreads=8))
    for k in (0, 7, 33):
        p, q = Pi[p_off[k]:p_off[k + 1]], Qi2[q_off[k]:q_off[k + 1]]
        assert ctx.dtw_distance_i32(dev(p), dev(q)).item() == oracle.dtw_i32(p, q)


def test_dtw_batched_workload_full_size_sampled(ctx):
    """The 4096-pair batched workload at full size; 40 sampled pairs against
    the oracle and the replica."""
    P, p_off, Q, q_off = workloads.batched()
    say("case: dtw batched workload, 4096 pairs")
    got = ctx.dtw_batch(dev(P), p_off, dev(Q), q_off, metric=oracle.SQEUCLIDEAN).cpu().numpy()
    assert ctx.last_errors() == 0
    idx = np.random.default_rng(216).choice(len(p_off) - 1, size=40, replace=False)
    ps, pl = p_off[:-1][idx], np.diff(p_off)[idx]
    qs, ql = q_off[:-1][idx], np.diff(q_off)[idx]
    want = oracle.dfd_pairs(P, ps, pl, Q, qs, ql, oracle.SQEUCLIDEAN, 8, measure="dtw")
    for r, k in enumerate(idx):
        assert abs(got[k] - want[r]) <= tol(pl[r], ql[r], 2, oracle.SQEUCLIDEAN) * want[r]
    for k in idx[:6]:
        p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
        assert got[k] == oracle.dtw_f32_replica(p, q, oracle.SQEUCLIDEAN)
