"""GPU parity for curves of 5 to 16 coordinates per point (the kernels of 8
and 16 coordinates, which hold zeros past the curves' own).

Bars as everywhere: float32 results bit-identical to the oracle's float32
replica (d2 = dx*dx, then fma(dk, dk, d2), or the sum / maximum of |dk|) and
within 2e-6 of the FP64 oracle; int32 and Levenshtein results exact.  A zero
coordinate adds an exact zero to every cell, so a curve padded with zero
coordinates must give the same bits on the wide kernels as on the kernel of
its own dimension: that pins the wide kernels against the narrow ones.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 2e-6


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


def pad(x, dim):
    out = np.zeros((x.shape[0], dim), dtype=x.dtype)
    out[:, :x.shape[1]] = x
    return out


def replica(P, p_off, Q, q_off, metric, dtw=False):
    f = oracle.dtw_f32_replica if dtw else oracle.dfd_f32_replica
    return np.array([f(P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]], metric) for k in range(len(p_off) - 1)],
                    dtype=np.float32)


@pytest.mark.parametrize("dim", [5, 8, 9, 12, 16])
def test_batch_matches_replica(ctx, dim):
    """Lengths 1 .. 900: one to eight bands of 128 (dim <= 8) or 64 rows,
    column curves shorter and longer than a group; the plan's own shape and
    every pair split into bands over waves (boundary rows through links)."""
    P, p_off, Q, q_off = workloads.random_pairs(900 + dim, 64, 1, 900, dim=dim)
    want0 = replica(P, p_off, Q, q_off, 0)
    for k in range(0, 64, 9):
        w = oracle.dfd(P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]], oracle.EUCLIDEAN, "rolling")
        assert abs(float(want0[k]) - w) <= TOL * w
    for metric in (0, 1):
        want = want0 if metric == 0 else replica(P, p_off, Q, q_off, metric)
        say(f"case: wide batch dim={dim} metric={metric}")
        got = ctx.batch(dev(P), p_off, dev(Q), q_off, metric=metric).cpu().numpy()
        assert ctx.last_errors() == 0
        assert ctx.last_launch()["rows_per_lane"] == (2 if dim <= 8 else 1)
        np.testing.assert_array_equal(got, want)
        ctx.set_split(1e-9)
        try:
            say(f"case: wide batch split dim={dim} metric={metric}")
            got = ctx.batch(dev(P), p_off, dev(Q), q_off, metric=metric).cpu().numpy()
            assert ctx.last_errors() == 0
        finally:
            ctx.set_split(0.0)
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("base", [1, 3, 4])
def test_zero_padding_is_exact(ctx, base):
    """Curves of `base` coordinates, zero-padded to 5 .. 16: the wide kernels
    give the narrow kernel's bits, for float32 (both Euclidean metrics,
    Manhattan, Chebyshev, DTW) and int32 coordinates."""
    P, p_off, Q, q_off = workloads.random_pairs(950 + base, 40, 1, 700, dim=base)
    Pi, pio, Qi, qio = workloads.random_pairs(960 + base, 30, 1, 500, dim=base, kind="int")
    ref = {m: ctx.batch(dev(P), p_off, dev(Q), q_off, metric=m).cpu().numpy() for m in (0, 1, 2, 3)}
    ref_dtw = {m: ctx.dtw_batch(dev(P), p_off, dev(Q), q_off, metric=m).cpu().numpy() for m in (0, 1)}
    ref_i = ctx.batch_i32(dev(Pi), pio, dev(Qi), qio).cpu().numpy()
    for dim in (5, 8, 11, 16):
        say(f"case: zero padding {base} -> {dim}")
        Pp, Qp = dev(pad(P, dim)), dev(pad(Q, dim))
        for m in (0, 1, 2, 3):
            np.testing.assert_array_equal(ctx.batch(Pp, p_off, Qp, q_off, metric=m).cpu().numpy(), ref[m])
        for m in (0, 1):
            np.testing.assert_array_equal(ctx.dtw_batch(Pp, p_off, Qp, q_off, metric=m).cpu().numpy(), ref_dtw[m])
        got = ctx.batch_i32(dev(pad(Pi, dim)), pio, dev(pad(Qi, dim)), qio).cpu().numpy()
        np.testing.assert_array_equal(got, ref_i)


@pytest.mark.parametrize("dim", [6, 13])
def test_single_pairs(ctx, dim):
    """Single pairs from one point to a long pair split into bands over
    waves (scratch registered by the binding); no pipelined kernel here."""
    rng = np.random.default_rng(970 + dim)
    for n, m in [(1, 1), (1, 300), (700, 5), (129, 127), (64, 65), (4000, 2500)]:
        p, q = workloads.walk(rng, n, dim), workloads.walk(rng, m, dim)
        say(f"case: wide single pair dim={dim} n={n} m={m}")
        got = ctx.distance(dev(p), dev(q)).item()
        assert ctx.last_errors() == 0
        assert ctx.last_launch()["pipelined"] == 0
        assert np.float32(got) == oracle.dfd_f32_replica(p, q, 0), (n, m)
        w = oracle.dfd(p, q, oracle.EUCLIDEAN, "rolling")
        assert abs(got - w) <= TOL * w


@pytest.mark.parametrize("dim", [7, 16])
def test_measures_and_int(ctx, dim):
    """DTW (squared and Euclidean cells), Manhattan and Chebyshev on float32
    against the replica; every int32 form exact (|x| < 2^15)."""
    P, p_off, Q, q_off = workloads.random_pairs(980 + dim, 30, 1, 600, dim=dim)
    say(f"case: wide dtw dim={dim} squared cells")
    got = ctx.dtw_batch(dev(P), p_off, dev(Q), q_off, metric=1).cpu().numpy()
    np.testing.assert_array_equal(got, replica(P, p_off, Q, q_off, 1, dtw=True))
    # Euclidean cells take the hardware square root (within 1 ulp) per cell:
    # the FP64 oracle within n + m + D + 3 float32 roundings
    say(f"case: wide dtw dim={dim} Euclidean cells")
    got = ctx.dtw_batch(dev(P), p_off, dev(Q), q_off, metric=0).cpu().numpy()
    for k in range(len(p_off) - 1):
        p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
        want = oracle.dtw(p, q, oracle.EUCLIDEAN)
        bound = (len(p) + len(q) + dim + 3) * 2.0 ** -24 * 1.01
        assert abs(float(got[k]) - want) <= bound * want, (k, float(got[k]), want)
    for metric in (oracle.MANHATTAN, oracle.CHEBYSHEV):
        say(f"case: wide metric dim={dim} metric={metric}")
        got = ctx.batch(dev(P), p_off, dev(Q), q_off, metric=metric).cpu().numpy()
        np.testing.assert_array_equal(got, replica(P, p_off, Q, q_off, metric))
        got = ctx.dtw_batch(dev(P), p_off, dev(Q), q_off, metric=metric).cpu().numpy()
        np.testing.assert_array_equal(got, replica(P, p_off, Q, q_off, metric, dtw=True))
    Qi, qoi, Di, doi = workloads.cross_int(seed=985 + dim, nq=4, ndb=25, length=200, dim=dim)
    for metric in (oracle.SQEUCLIDEAN, oracle.MANHATTAN, oracle.CHEBYSHEV):
        say(f"case: wide int cross dim={dim} metric={metric}")
        got = ctx.cross_i32(dev(Qi), qoi, dev(Di), doi, metric=metric).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.dfd_cross_i32(Qi, qoi, Di, doi, nthreads=8, metric=metric))
        got = ctx.dtw_cross_i32(dev(Qi), qoi, dev(Di), doi, metric=metric).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.dtw_cross_i32(Qi, qoi, Di, doi, nthreads=8, metric=metric))
    a, b = Qi[qoi[1]:qoi[2]], Di[doi[3]:doi[4]]
    assert ctx.distance_i32(dev(a), dev(b)).item() == oracle.dfd_i32(a, b)


@pytest.mark.parametrize("dim", [6, 16])
def test_levenshtein(ctx, dim):
    """Symbols of `dim` int32 coordinates: two symbols are equal when every
    coordinate is (few distinct values, so that equal symbols are common)."""
    rng = np.random.default_rng(990 + dim)
    ps, qs = [], []
    for k in range(40):
        n, m = int(rng.integers(1, 500)), int(rng.integers(1, 500))
        ps.append(rng.integers(0, 2, size=(n, dim)).astype(np.int32))
        qs.append(rng.integers(0, 2, size=(m, dim)).astype(np.int32))
        if k % 3 == 0:
            qs[-1][: min(n, m) // 2] = ps[-1][: min(n, m) // 2]
    P, p_off = workloads.concat(ps)
    Q, q_off = workloads.concat(qs)
    say(f"case: wide levenshtein dim={dim}")
    got = ctx.levenshtein_batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    assert ctx.last_errors() == 0
    np.testing.assert_array_equal(got, oracle.lev_batch(P, p_off, Q, q_off, nthreads=8))
    assert ctx.levenshtein(dev(ps[3]), dev(qs[3])).item() == oracle.lev(ps[3], qs[3])


@pytest.mark.parametrize("dim", [10])
def test_cross(ctx, dim):
    rng = np.random.default_rng(995)
    qs = [workloads.walk(rng, int(L), dim) for L in rng.integers(1, 900, size=5)]
    db = [workloads.walk(rng, int(L), dim) for L in rng.integers(1, 1200, size=70)]
    Qs, qo = workloads.concat(qs)
    DB, do = workloads.concat(db)
    say(f"case: wide cross dim={dim}")
    got = ctx.cross(dev(Qs), qo, dev(DB), do).cpu().numpy()
    for i in range(5):
        want = np.array([oracle.dfd_f32_replica(qs[i], db[c], 0) for c in range(70)], dtype=np.float32)
        np.testing.assert_array_equal(got[i], want)


@pytest.mark.parametrize("dim", [5, 12])
def test_decider_and_knn(ctx, dim):
    """The early-abandoning sweep (its own kernels of 8 and 16 coordinates):
    the decider gives where(delta <= eps, delta, +inf) and the search the k
    smallest (delta, index) pairs, bit for bit."""
    P, p_off, Q, q_off = workloads.random_pairs(1000 + dim, 60, 1, 700, dim=dim)
    want = replica(P, p_off, Q, q_off, 0)
    for qt in (0.0, 0.3, 0.7, 1.0):
        eps = float(np.quantile(want, qt))
        say(f"case: wide decider dim={dim} eps=quantile {qt}")
        got = ctx.decide_batch(dev(P), p_off, dev(Q), q_off, eps).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.decide(want, np.float32(eps)))
    rng = np.random.default_rng(1010 + dim)
    db = [workloads.walk(rng, int(L), dim) for L in rng.integers(8, 600, size=120)]
    DB, do = workloads.concat(db)
    queries = [workloads.walk(rng, int(L), dim) for L in (30, 200, 450)]
    Qs, qo = workloads.concat(queries)
    say(f"case: wide knn dim={dim}")
    gi, gd = ctx.knn_batch(dev(Qs), qo, dev(DB), do, 7)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    for i, q in enumerate(queries):
        vals = np.array([oracle.dfd_f32_replica(q, c, 0) for c in db], dtype=np.float32)
        want_i, want_d = oracle.knn(vals, 7)
        np.testing.assert_array_equal(gd[i], want_d)
        np.testing.assert_array_equal(gi[i], want_i)


def test_serving(ctx):
    """A server over a database of 9-coordinate curves: each query's results
    equal ffd_cross's, bit for bit, alone and submitted together."""
    from paper_2404_05708_amd import ffd
    dim = 9
    rng = np.random.default_rng(1020)
    db = [workloads.walk(rng, int(L), dim) for L in rng.integers(8, 900, size=200)]
    DB, do = workloads.concat(db)
    DBd = dev(DB)
    qs = [workloads.walk(rng, int(L), dim) for L in (5, 70, 300, 1500)]
    database = ffd.Database(ctx, DBd, do)
    srv = ffd.Server(database, max_slots=4, max_query=2048)
    try:
        say("case: wide serving, queries alone")
        alone = [srv.wait(srv.submit(q)).copy() for q in qs]
        say("case: wide serving, queries together")
        tickets = [srv.submit(q) for q in qs]
        mix = [srv.wait(t).copy() for t in tickets]
    finally:
        srv.close()
        database.close()
    Qs, qo = workloads.concat(qs)
    cross = ctx.cross(dev(Qs), qo, DBd, do).cpu().numpy()
    for i in range(len(qs)):
        np.testing.assert_array_equal(alone[i], cross[i])
        np.testing.assert_array_equal(mix[i], cross[i])
    want = np.array([oracle.dfd_f32_replica(qs[1], c, 0) for c in db], dtype=np.float32)
    np.testing.assert_array_equal(cross[1], want)
