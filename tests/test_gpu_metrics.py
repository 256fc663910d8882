"""GPU parity of the Manhattan and Chebyshev ground distances, for the
Frechet distance and DTW, through the C ABI.

Bars: float32 results bit-identical to the float32 replica (the cell value
is |d0| then + |dk| or max(., |dk|) in coordinate order, the recurrence
only selects, or adds in the order the recurrence fixes) and within a
relative 2e-6 (Frechet) or (n + m + 2 D + 2) 2^-24 (DTW) of the FP64 oracle;
int32 results bit-exact; every launch shape and the batch, cross and
single-pair forms give the same bits.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

MET = (oracle.MANHATTAN, oracle.CHEBYSHEV)


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


def check(got, p, q, metric, dtw):
    n, D = p.shape
    m = q.shape[0]
    if dtw:
        want = oracle.dtw(p, q, metric)
        tol = (n + m + 2 * D + 2) * 2.0 ** -24 * 1.01
        rep = oracle.dtw_f32_replica(p, q, metric)
    else:
        want = oracle.dfd(p, q, metric, "rolling")
        tol = 2e-6
        rep = oracle.dfd_f32_replica(p, q, metric)
    assert abs(float(got) - want) <= tol * want, (n, m, D, metric, dtw, float(got), want)
    assert np.float32(got) == rep, (n, m, D, metric, dtw)


@pytest.mark.parametrize("R", [0, 1, 2, 4, 8])
def test_random_shapes(ctx, R):
    rng = np.random.default_rng(300 + R)
    ctx.set_tuning(R, 0)
    try:
        for it in range(10):
            n, m, D = int(rng.integers(1, 700)), int(rng.integers(1, 700)), int(rng.integers(1, 5))
            p, q = workloads.walk(rng, n, D), workloads.walk(rng, m, D)
            for metric in MET:
                say(f"case: metrics R={R} n={n} m={m} D={D} metric={metric}")
                check(ctx.distance(dev(p), dev(q), metric=metric).item(), p, q, metric, False)
                check(ctx.dtw_distance(dev(p), dev(q), metric=metric).item(), p, q, metric, True)
    finally:
        ctx.set_tuning(0, 0)


def test_batch_cross_pairs_and_split_agree(ctx):
    P, p_off, Q, q_off = workloads.random_pairs(310, 120, 1, 2600, dim=3)
    for metric in MET:
        for dtw in (False, True):
            fn = ctx.dtw_batch if dtw else ctx.batch
            say(f"case: metrics batch metric={metric} dtw={dtw}")
            base = fn(dev(P), p_off, dev(Q), q_off, metric=metric).cpu().numpy()
            for k in range(0, len(p_off) - 1, 20):
                p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
                check(base[k], p, q, metric, dtw)
                one = (ctx.dtw_distance if dtw else ctx.distance)(dev(p), dev(q), metric=metric).item()
                assert one == base[k]
            ctx.set_tuning(2, 0)
            ctx.set_split(1e-9)
            try:
                got = fn(dev(P), p_off, dev(Q), q_off, metric=metric).cpu().numpy()
                assert ctx.last_errors() == 0
            finally:
                ctx.set_split(0.0)
                ctx.set_tuning(0, 0)
            np.testing.assert_array_equal(got, base)
    Qs, qo = workloads.concat([P[p_off[k]:p_off[k + 1]] for k in range(3)])
    DB, do = workloads.concat([Q[q_off[k]:q_off[k + 1]] for k in range(25)])
    for metric in MET:
        say(f"case: metrics cross metric={metric}")
        cr = ctx.cross(dev(Qs), qo, dev(DB), do, metric=metric).cpu().numpy()
        cw = ctx.dtw_cross(dev(Qs), qo, dev(DB), do, metric=metric).cpu().numpy()
        for i in range(3):
            for k in range(0, 25, 6):
                a, b = Qs[qo[i]:qo[i + 1]], DB[do[k]:do[k + 1]]
                check(cr[i, k], a, b, metric, False)
                check(cw[i, k], a, b, metric, True)


def test_int_exact(ctx):
    Qi, qoi, Di, doi = workloads.cross_int(seed=311, nq=5, ndb=40, length=300, dim=3)
    for metric in MET:
        say(f"case: metrics int cross metric={metric}")
        got = ctx.cross_i32(dev(Qi), qoi, dev(Di), doi, metric=metric).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.dfd_cross_i32(Qi, qoi, Di, doi, nthreads=8, metric=metric))
        got = ctx.dtw_cross_i32(dev(Qi), qoi, dev(Di), doi, metric=metric).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.dtw_cross_i32(Qi, qoi, Di, doi, nthreads=8, metric=metric))
        bi = ctx.batch_i32(dev(Qi), qoi, dev(Di), doi[:6], metric=metric).cpu().numpy()
        np.testing.assert_array_equal(bi, oracle.dfd_batch_i32(Qi, qoi, Di, doi[:6], nthreads=4, metric=metric))
        a, b = Qi[qoi[1]:qoi[2]], Di[doi[7]:doi[8]]
        assert ctx.distance_i32(dev(a), dev(b), metric=metric).item() == oracle.dfd_i32(a, b, metric)
        assert ctx.dtw_distance_i32(dev(a), dev(b), metric=metric).item() == oracle.dtw_i32(a, b, metric)


def test_long_pairs(ctx):
    """Long single pairs split over waves (no LDS-ring pipeline for these
    kernels) and column curves longer than the LDS hand-off row."""
    rng = np.random.default_rng(312)
    for n, m in [(3000, 2000), (700, 9000)]:
        p, q = workloads.walk(rng, n, 2), workloads.walk(rng, m, 2)
        for metric in MET:
            say(f"case: metrics long pair n={n} m={m} metric={metric}")
            check(ctx.distance(dev(p), dev(q), metric=metric).item(), p, q, metric, False)
            assert ctx.last_errors() == 0
            check(ctx.dtw_distance(dev(p), dev(q), metric=metric).item(), p, q, metric, True)
            assert ctx.last_errors() == 0
