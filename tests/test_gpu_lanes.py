"""GPU parity of the one-pair-per-lane kernel (batches of short pairs).

The lane kernel evaluates every cell as the streaming kernels do and takes
the Euclidean root once per pair, so its results must equal the streaming
kernel's (forced with a rows-per-lane setting, which keeps the job-table
plan) bit for bit, for every pair; a sample is also checked against the
oracle's float32 replica and the FP64 oracle (2e-6), and the int32 path
against the int64 oracle for every pair.  Lengths cover the column classes
(multiples of 8 up to 64), their boundaries, single points and both
orientations.
"""
import sys

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu
TOL = 2e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ffdmod(gpu):
    from paper_2404_05708_amd import ffd
    return ffd


@pytest.fixture(scope="module")
def ctx(ffdmod):
    c = ffdmod.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def short_pairs(seed, count, lo, hi, dim, kind="walk"):
    """count pairs with lengths uniform in [lo, hi], plus the class
    boundaries and single points; random walks (float32) or int32 in
    [-2^15, 2^15).  Returns P, p_off, Q, q_off."""
    rng = np.random.default_rng(seed)
    edge = [(1, 1), (1, hi), (hi, 1), (16, 16), (17, 16), (16, 17), (32, 33), (33, 32), (64, 64), (63, 64),
            (5, 64), (64, 5)]
    edge = [(a, b) for a, b in edge if a <= hi and b <= hi]
    n = np.concatenate([rng.integers(lo, hi + 1, size=count), [e[0] for e in edge]]).astype(np.int64)
    m = np.concatenate([rng.integers(lo, hi + 1, size=count), [e[1] for e in edge]]).astype(np.int64)
    p_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    q_off = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)

    def curves(off):
        total = int(off[-1])
        if kind == "int":
            return rng.integers(-(1 << 15), 1 << 15, size=(total, dim), dtype=np.int32)
        x = np.cumsum(rng.standard_normal((total, dim)), axis=0)
        starts = np.repeat(x[off[:-1]] - rng.standard_normal((len(off) - 1, dim)), np.diff(off), axis=0)
        return (x - starts).astype(np.float32)  # a walk per curve, starting near 0

    return curves(p_off), p_off, curves(q_off), q_off


@pytest.mark.parametrize("dim,hi", [(1, 64), (2, 64), (3, 32), (4, 32), (2, 16)])
def test_lanes_equal_streaming_kernel(ctx, dim, hi):
    P, p_off, Q, q_off = short_pairs(500 + dim + hi, 150000, 1, hi, dim)
    Pd, Qd = dev(P), dev(Q)
    npairs = len(p_off) - 1
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(npairs, size=300, replace=False))
    sample = np.unique(np.concatenate([sample, np.arange(npairs - 12, npairs)]))  # the edge cases
    for metric in (0, 1):
        say(f"case: lanes dim={dim} hi={hi} metric={metric}")
        got = ctx.batch(Pd, p_off, Qd, q_off, metric=metric).cpu().numpy()
        info = ctx.last_launch()
        assert info["per_lane"] == 1 and info["rows_per_lane"] == 0, info
        assert ctx.last_errors() == 0
        ctx.set_tuning(1, 0)  # the job-table plan of the streaming kernel
        try:
            say(f"case: streaming kernel on the same pairs dim={dim} metric={metric}")
            ref = ctx.batch(Pd, p_off, Qd, q_off, metric=metric).cpu().numpy()
            assert ctx.last_launch()["per_lane"] == 0
        finally:
            ctx.set_tuning(0, 0)
        np.testing.assert_array_equal(got, ref)
        for k in sample:
            p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
            assert got[k] == oracle.dfd_f32_replica(p, q, metric), (k, len(p), len(q))
        if metric == 0:
            want = oracle.dfd_pairs(P, p_off[:-1][sample], np.diff(p_off)[sample], Q, q_off[:-1][sample],
                                    np.diff(q_off)[sample], 0, 8)
            assert np.all(np.abs(got[sample] - want) <= TOL * want)


@pytest.mark.parametrize("dim,hi", [(1, 64), (3, 32)])
def test_lanes_manhattan_chebyshev(ctx, ffdmod, dim, hi):
    """The Frechet distance on Manhattan and Chebyshev cells, one pair per
    lane: the streaming kernel's bits for every pair, the replica's on a
    sample."""
    P, p_off, Q, q_off = short_pairs(550 + dim, 150000, 1, hi, dim)
    Pd, Qd = dev(P), dev(Q)
    sample = np.arange(0, len(p_off) - 1, 997)
    for metric in (ffdmod.FFD_MANHATTAN, ffdmod.FFD_CHEBYSHEV):
        say(f"case: lanes dim={dim} metric={metric}")
        got = ctx.batch(Pd, p_off, Qd, q_off, metric=metric).cpu().numpy()
        assert ctx.last_launch()["per_lane"] == 1
        ctx.set_tuning(1, 0)
        try:
            ref = ctx.batch(Pd, p_off, Qd, q_off, metric=metric).cpu().numpy()
        finally:
            ctx.set_tuning(0, 0)
        np.testing.assert_array_equal(got, ref)
        for k in sample:
            p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
            assert got[k] == oracle.dfd_f32_replica(p, q, metric), k
    Pi, pio, Qi, qio = short_pairs(560 + dim, 150000, 1, 16, dim, kind="int")
    for metric in (ffdmod.FFD_MANHATTAN, ffdmod.FFD_CHEBYSHEV):
        say(f"case: lanes int32 dim={dim} metric={metric}")
        got = ctx.batch_i32(dev(Pi), pio, dev(Qi), qio, metric=metric).cpu().numpy()
        assert ctx.last_launch()["per_lane"] == 1
        np.testing.assert_array_equal(got, oracle.dfd_batch_i32(Pi, pio, Qi, qio, nthreads=8, metric=metric))


@pytest.mark.parametrize("dim,hi", [(1, 64), (2, 64), (3, 32)])
def test_lanes_dtw(ctx, ffdmod, dim, hi):
    """DTW one pair per lane (sums: the result read at the column curve's own
    last column, no repeated row): the streaming kernel's bits for every pair
    on every cell, the replica's on a sample; int32 exact."""
    P, p_off, Q, q_off = short_pairs(570 + dim, 150000, 1, hi, dim)
    Pd, Qd = dev(P), dev(Q)
    sample = np.arange(0, len(p_off) - 1, 1499)
    sample = np.unique(np.concatenate([sample, np.arange(len(p_off) - 13, len(p_off) - 1)]))
    for metric in (ffdmod.FFD_SQEUCLIDEAN, ffdmod.FFD_EUCLIDEAN, ffdmod.FFD_MANHATTAN, ffdmod.FFD_CHEBYSHEV):
        say(f"case: lanes dtw dim={dim} metric={metric}")
        got = ctx.dtw_batch(Pd, p_off, Qd, q_off, metric=metric).cpu().numpy()
        assert ctx.last_launch()["per_lane"] == 1
        ctx.set_tuning(1, 0)
        try:
            ref = ctx.dtw_batch(Pd, p_off, Qd, q_off, metric=metric).cpu().numpy()
            assert ctx.last_launch()["per_lane"] == 0
        finally:
            ctx.set_tuning(0, 0)
        np.testing.assert_array_equal(got, ref)
        if metric != ffdmod.FFD_EUCLIDEAN:  # the replica takes the correctly rounded root per cell
            for k in sample:
                p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
                assert got[k] == oracle.dtw_f32_replica(p, q, metric), (k, len(p), len(q))
    Pi, pio, Qi, qio = short_pairs(580 + dim, 150000, 1, 16, dim, kind="int")
    say(f"case: lanes dtw int32 dim={dim}")
    got = ctx.dtw_batch_i32(dev(Pi), pio, dev(Qi), qio).cpu().numpy()
    assert ctx.last_launch()["per_lane"] == 1
    np.testing.assert_array_equal(got, oracle.dtw_batch_i32(Pi, pio, Qi, qio, nthreads=8))


@pytest.mark.parametrize("dim,alphabet", [(1, 4), (1, 26), (2, 3)])
def test_lanes_levenshtein(ctx, dim, alphabet):
    """Levenshtein on short symbol sequences, one pair per lane (and query
    set x database): the streaming kernel's values for every pair, and the
    int64 oracle's."""
    rng = np.random.default_rng(590 + alphabet)
    count = 150000
    n = np.concatenate([rng.integers(1, 65, size=count), [1, 64, 64, 1, 63]])
    m = np.concatenate([rng.integers(1, 65, size=count), [1, 64, 1, 64, 64]])
    p_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    q_off = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    P = rng.integers(0, alphabet, size=(int(p_off[-1]), dim)).astype(np.int32)
    Q = rng.integers(0, alphabet, size=(int(q_off[-1]), dim)).astype(np.int32)
    Pd, Qd = dev(P), dev(Q)
    say(f"case: lanes levenshtein dim={dim} alphabet={alphabet}")
    got = ctx.levenshtein_batch(Pd, p_off, Qd, q_off).cpu().numpy()
    assert ctx.last_launch()["per_lane"] == 1
    ctx.set_tuning(1, 0)
    try:
        ref = ctx.levenshtein_batch(Pd, p_off, Qd, q_off).cpu().numpy()
        assert ctx.last_launch()["per_lane"] == 0
    finally:
        ctx.set_tuning(0, 0)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(got, oracle.lev_batch(P, p_off, Q, q_off, nthreads=8))
    say(f"case: lanes levenshtein cross dim={dim}")
    Qs, qo = P[:p_off[300]], p_off[:301]
    DB, do = Q[:q_off[500]], q_off[:501]
    cr = ctx.levenshtein_cross(dev(Qs), qo, dev(DB), do).cpu().numpy()
    assert ctx.last_launch()["per_lane"] == 1
    np.testing.assert_array_equal(cr, oracle.lev_cross(Qs, qo, DB, do, nthreads=8))


@pytest.mark.parametrize("dim,hi", [(2, 32), (4, 16)])
def test_lanes_int_exact(ctx, dim, hi):
    P, p_off, Q, q_off = short_pairs(600 + dim, 150000, 1, hi, dim, kind="int")
    say(f"case: lanes int32 dim={dim} hi={hi}")
    got = ctx.batch_i32(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    assert ctx.last_launch()["per_lane"] == 1
    np.testing.assert_array_equal(got, oracle.dfd_batch_i32(P, p_off, Q, q_off, nthreads=8))


def test_lanes_graph_replay_and_noalloc(ctx, ffdmod):
    """A batch on the lane kernel recorded into a graph replays the eager
    bits; the no-allocation entry point gives them too."""
    P, p_off, Q, q_off = short_pairs(700, 150000, 1, 64, 2)
    Pd, Qd = dev(P), dev(Q)
    out = torch.empty(len(p_off) - 1, dtype=torch.float32, device="cuda:0")
    ws = torch.empty(ctx.workspace_size(ffdmod.FFD_OP_BATCH, p_off, q_off, 2), dtype=torch.uint8, device="cuda:0")
    say("case: lanes, eager call")
    ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws)
    torch.cuda.synchronize()
    assert ctx.last_launch()["per_lane"] == 1
    eager = out.clone()
    g = torch.cuda.CUDAGraph()
    say("case: lanes, capture")
    with torch.cuda.graph(g):
        ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws)
    for k in range(3):
        say(f"case: lanes, replay {k}")
        out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k
    say("case: lanes, no-allocation entry point")
    got = ctx.batch_noalloc(Pd, p_off, Qd, q_off)
    torch.cuda.synchronize()
    assert torch.equal(got, eager)


def test_lanes_with_long_pairs(ctx, ffdmod):
    """Short and long pairs in one batch: the short ones one per lane, the
    long ones on the streaming kernel in a launch after them; every result
    equals the streaming kernel's for the whole batch, a sample the
    replica's; graph replay gives the eager bits."""
    rng = np.random.default_rng(710)
    n = np.concatenate([rng.integers(1, 65, size=150000), rng.integers(300, 1501, size=800)])
    m = np.concatenate([rng.integers(1, 65, size=150000), rng.integers(300, 1501, size=800)])
    perm = rng.permutation(len(n))
    n, m = n[perm], m[perm]
    p_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    q_off = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    P = np.cumsum(rng.standard_normal((int(p_off[-1]), 2)), axis=0).astype(np.float32)
    Q = (P[np.minimum(np.arange(int(q_off[-1])), len(P) - 1)] + rng.standard_normal((int(q_off[-1]), 2))
         ).astype(np.float32)
    Pd, Qd = dev(P), dev(Q)
    out = torch.empty(len(n), dtype=torch.float32, device="cuda:0")
    ws = torch.empty(ctx.workspace_size(ffdmod.FFD_OP_BATCH, p_off, q_off, 2), dtype=torch.uint8, device="cuda:0")
    say("case: lanes with long pairs, eager call")
    ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws)
    torch.cuda.synchronize()
    info = ctx.last_launch()
    assert info["per_lane"] == 1 and info["rows_per_lane"] > 0, info
    assert ctx.last_errors() == 0
    got = out.cpu().numpy()
    ctx.set_tuning(2, 0)
    try:
        say("case: the whole batch on the streaming kernel")
        ref = ctx.batch(Pd, p_off, Qd, q_off).cpu().numpy()
        assert ctx.last_launch()["per_lane"] == 0
    finally:
        ctx.set_tuning(0, 0)
    np.testing.assert_array_equal(got, ref)
    longs = np.nonzero(np.minimum(n, m) > 64)[0]
    for k in np.concatenate([longs[:20], np.arange(0, len(n), 5003)]):
        p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
        assert got[k] == oracle.dfd_f32_replica(p, q, 0), (k, len(p), len(q))
    # a capture needs the same call's plan in the workspace: the eager call again
    ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("case: lanes with long pairs, capture and replays")
    with torch.cuda.graph(g):
        ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws)
    for k in range(3):
        out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert ctx.last_errors() == 0
        np.testing.assert_array_equal(out.cpu().numpy(), got)


def test_lanes_cross(ctx, ffdmod):
    """Queries x database of short curves, one (query, curve) pair per lane:
    the streaming kernel's bits for every pair, Frechet and DTW, float32 and
    int32 (exact against the oracle)."""
    rng = np.random.default_rng(720)
    qs = [np.cumsum(rng.standard_normal((int(L), 2)), axis=0).astype(np.float32) for L in rng.integers(1, 49, 400)]
    db = [np.cumsum(rng.standard_normal((int(L), 2)), axis=0).astype(np.float32) for L in rng.integers(1, 49, 500)]
    qo = np.concatenate([[0], np.cumsum([len(q) for q in qs])]).astype(np.int64)
    do = np.concatenate([[0], np.cumsum([len(c) for c in db])]).astype(np.int64)
    Qd, Dd = dev(np.concatenate(qs)), dev(np.concatenate(db))
    for dtw in (False, True):
        say(f"case: lanes cross dtw={dtw}")
        call = ctx.dtw_cross if dtw else ctx.cross
        got = call(Qd, qo, Dd, do, metric=ffdmod.FFD_SQEUCLIDEAN).cpu().numpy()
        assert ctx.last_launch()["per_lane"] == 1
        ctx.set_tuning(1, 0)
        try:
            ref = call(Qd, qo, Dd, do, metric=ffdmod.FFD_SQEUCLIDEAN).cpu().numpy()
            assert ctx.last_launch()["per_lane"] == 0
        finally:
            ctx.set_tuning(0, 0)
        np.testing.assert_array_equal(got, ref)
        f = oracle.dtw_f32_replica if dtw else oracle.dfd_f32_replica
        for i in (0, 17, 399):
            for c in (0, 250, 499):
                assert got.reshape(400, 500)[i, c] == f(qs[i], db[c], ffdmod.FFD_SQEUCLIDEAN), (i, c)
    Qi, qoi, Di, doi = workloads_cross_int(rng)
    say("case: lanes cross int32")
    got = ctx.cross_i32(dev(Qi), qoi, dev(Di), doi).cpu().numpy()
    assert ctx.last_launch()["per_lane"] == 1
    np.testing.assert_array_equal(got, oracle.dfd_cross_i32(Qi, qoi, Di, doi, nthreads=8))


def workloads_cross_int(rng):
    lq, ld = rng.integers(1, 33, 300), rng.integers(1, 33, 600)
    qo = np.concatenate([[0], np.cumsum(lq)]).astype(np.int64)
    do = np.concatenate([[0], np.cumsum(ld)]).astype(np.int64)
    Qi = rng.integers(-(1 << 15), 1 << 15, size=(int(qo[-1]), 2), dtype=np.int32)
    Di = rng.integers(-(1 << 15), 1 << 15, size=(int(do[-1]), 2), dtype=np.int32)
    return Qi, qo, Di, do


def test_kernel_timing(ctx):
    # the library's event pair brackets the kernels alone: no longer than the
    # whole call on the same stream, one record per launch, none when off
    P, p_off, Q, q_off = short_pairs(611, 60000, 8, 64, 2)
    Pd, Qd = dev(P), dev(Q)
    out = torch.empty(len(p_off) - 1, dtype=torch.float32, device="cuda:0")
    ctx.batch(Pd, p_off, Qd, q_off, out=out)  # plan cached
    for forced in (False, True):
        if forced:
            ctx.set_tuning(1, 0)  # the streaming kernel's job-table plan
        try:
            say(f"case: kernel timing forced_stream={forced}")
            ctx.batch(Pd, p_off, Qd, q_off, out=out)
            torch.cuda.synchronize()
            ctx.set_kernel_timing(True)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(5):
                ctx.batch(Pd, p_off, Qd, q_off, out=out)
            b.record()
            torch.cuda.synchronize()
            ms, n = ctx.kernel_time()
            assert n == 5 and ctx.last_launch()["per_lane"] == (0 if forced else 1)
            assert 0 < ms <= a.elapsed_time(b) * 1.001 + 0.01, (ms, a.elapsed_time(b))
            assert ctx.kernel_time() == (0.0, 0)  # read clears the record
            ctx.set_kernel_timing(False)
            ctx.batch(Pd, p_off, Qd, q_off, out=out)
            assert ctx.kernel_time() == (0.0, 0)
        finally:
            ctx.set_kernel_timing(False)
            ctx.set_tuning(0, 0)
