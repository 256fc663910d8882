"""GPU parity: the HIP library through the C ABI against the CPU oracle.

Bars: float32 results within a relative error of 2e-6 of the FP64 oracle
(exactly 0 where the oracle is 0); int32 results bit-exact.  Where the
float32 evaluation order is fixed (d2 = dx*dx, then fma(dk, dk, d2)), the GPU
must also reproduce the float replica bit for bit: the recurrence only
selects values, so any disagreement would mean a wrong cell was selected.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
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


def rel_ok(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return np.all(np.abs(got - want) <= TOL * np.abs(want))


def test_dpp_lane_shift_semantics(ctx):
    """A 64-lane single band exercises the wave-wide lane shift: rows of every
    lane must see the row above, so any wrong neighbour changes the value."""
    say("case: dpp shift, n=64*4, R=4")
    rng = np.random.default_rng(5)
    p = workloads.walk(rng, 256, 2)
    q = workloads.walk(rng, 300, 2)
    ctx.set_tuning(4, 0)
    got = ctx.distance(dev(p), dev(q)).item()
    ctx.set_tuning(0, 0)
    assert got == oracle.dfd_f32_replica(p, q)


def test_plain_pair_workload(ctx):
    say("case: plain pair 512 x 384")
    g = json.load(open(os.path.join(HERE, "golden", "expected.json")))["plain_pair"]
    p, q = workloads.plain_pair()
    got = ctx.distance(dev(p), dev(q)).item()
    assert rel_ok(got, g["euclidean"])
    assert got == oracle.dfd_f32_replica(p, q)
    got_sq = ctx.distance(dev(p), dev(q), metric=1).item()
    assert rel_ok(got_sq, g["sqeuclidean"])
    assert got_sq == oracle.dfd_f32_replica(p, q, 1)


@pytest.mark.parametrize("R", [0, 1, 2, 4, 8])
def test_random_shapes_all_dims(ctx, R):
    rng = np.random.default_rng(100 + R)
    ctx.set_tuning(R, 0)
    try:
        for it in range(24):
            D = int(rng.integers(1, 5))
            n = int(rng.integers(1, 700))
            m = int(rng.integers(1, 700))
            metric = int(rng.integers(0, 2))
            say(f"case: random R={R} it={it} n={n} m={m} D={D} metric={metric}")
            p = workloads.walk(rng, n, D)
            q = workloads.walk(rng, m, D)
            got = ctx.distance(dev(p), dev(q), metric=metric).item()
            assert got == oracle.dfd_f32_replica(p, q, metric), (n, m, D, metric)
            assert rel_ok(got, oracle.dfd(p, q, metric, "rolling"))
    finally:
        ctx.set_tuning(0, 0)


def test_edge_cases(ctx):
    rng = np.random.default_rng(9)
    for n, m in [(1, 1), (1, 5), (5, 1), (1, 700), (700, 1), (2, 2), (63, 65), (64, 64), (65, 63),
                 (257, 3), (3, 1025)]:
        say(f"case: edge n={n} m={m}")
        p = workloads.walk(rng, n, 2)
        q = workloads.walk(rng, m, 2)
        got = ctx.distance(dev(p), dev(q)).item()
        assert got == oracle.dfd_f32_replica(p, q)
        assert rel_ok(got, oracle.dfd(p, q))
    say("case: identical curves")
    p = workloads.walk(rng, 333, 3)
    assert ctx.distance(dev(p), dev(p)).item() == 0.0
    say("case: translated copy")
    q = workloads.paper_walk(rng, 200, 2)
    assert ctx.distance(dev(q + np.float32([3, 4])), dev(q)).item() == 5.0


def test_invariances_bit_exact(ctx):
    rng = np.random.default_rng(10)
    for it in range(6):
        n, m = int(rng.integers(1, 900)), int(rng.integers(1, 900))
        say(f"case: invariances n={n} m={m}")
        p = workloads.walk(rng, n, 2)
        q = workloads.walk(rng, m, 2)
        d = ctx.distance(dev(p), dev(q)).item()
        assert ctx.distance(dev(q), dev(p)).item() == d
        assert ctx.distance(dev(p[::-1].copy()), dev(q[::-1].copy())).item() == d
        pad = np.concatenate([p, np.repeat(p[-1:], 37, axis=0)])
        assert ctx.distance(dev(pad), dev(q)).item() == d


def test_paper_walks_are_bit_exact(ctx):
    """{-1,0,1} walks: every float32 squared distance is an exact integer, so
    the GPU result is the float32 rounding of the FP64 oracle."""
    rng = np.random.default_rng(11)
    for it in range(6):
        n, m = int(rng.integers(1, 1024)), int(rng.integers(1, 1024))
        say(f"case: paper walk n={n} m={m}")
        p = workloads.paper_walk(rng, n)
        q = workloads.paper_walk(rng, m)
        assert ctx.distance(dev(p), dev(q)).item() == np.float32(oracle.dfd(p, q))


def test_int_pairs_exact(ctx):
    rng = np.random.default_rng(12)
    for it in range(12):
        D = int(rng.integers(1, 5))
        n, m = int(rng.integers(1, 600)), int(rng.integers(1, 600))
        say(f"case: int n={n} m={m} D={D}")
        p = rng.integers(-(1 << 15), 1 << 15, size=(n, D), dtype=np.int32)
        q = rng.integers(-(1 << 15), 1 << 15, size=(m, D), dtype=np.int32)
        got = ctx.distance_i32(dev(p), dev(q)).item()
        assert got == oracle.dfd_i32(p, q)


def test_batch_small_and_ragged(ctx):
    for seed, npairs, lo, hi in [(20, 50, 1, 300), (21, 200, 1, 80), (22, 30, 500, 2100)]:
        say(f"case: batch seed={seed} npairs={npairs} lengths [{lo},{hi}]")
        P, p_off, Q, q_off = workloads.random_pairs(seed, npairs, lo, hi, dim=2)
        got = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
        want = oracle.dfd_batch(P, p_off, Q, q_off, nthreads=8)
        assert rel_ok(got, want)
        for k in range(npairs):
            assert got[k] == oracle.dfd_f32_replica(P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]])


def test_batch_equals_plain_and_tuning_invariant(ctx):
    P, p_off, Q, q_off = workloads.random_pairs(23, 40, 1, 1500, dim=3)
    say("case: batch vs plain, 40 pairs D=3")
    base = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    for k in range(40):
        one = ctx.distance(dev(P[p_off[k]:p_off[k + 1]]), dev(Q[q_off[k]:q_off[k + 1]])).item()
        assert one == base[k]
    for R in (1, 2, 4, 8):
        for W in (1, 2):
            say(f"case: tuning R={R} W={W}")
            ctx.set_tuning(R, W)
            try:
                got = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
            finally:
                ctx.set_tuning(0, 0)
            np.testing.assert_array_equal(got, base)


def test_batch_int_exact(ctx):
    say("case: batch int")
    P, p_off, Q, q_off = workloads.random_pairs(24, 60, 1, 700, dim=2, kind="int")
    got = ctx.batch_i32(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.dfd_batch_i32(P, p_off, Q, q_off, nthreads=8))


def test_cross_small(ctx):
    say("case: cross float")
    rng = np.random.default_rng(25)
    Qs, qo = workloads.concat([workloads.walk(rng, int(rng.integers(1, 700)), 2) for _ in range(6)])
    DB, do = workloads.concat([workloads.walk(rng, int(rng.integers(1, 400)), 2) for _ in range(37)])
    got = ctx.cross(dev(Qs), qo, dev(DB), do).cpu().numpy()
    want = oracle.dfd_cross(Qs, qo, DB, do, nthreads=8)
    assert rel_ok(got, want)
    say("case: cross int")
    Qi, qoi, Di, doi = workloads.cross_int(seed=26, nq=7, ndb=50, length=97)
    got = ctx.cross_i32(dev(Qi), qoi, dev(Di), doi).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.dfd_cross_i32(Qi, qoi, Di, doi, nthreads=8))


def test_batched_workload_full_size(ctx):
    """All 4096 pairs in the launch configuration the benchmark times, every
    output against the FP64 oracle (the rolling form on 16 threads), plus
    the stored sample and the end-point lower bound."""
    say("case: batched workload 4096 pairs")
    g = json.load(open(os.path.join(HERE, "golden", "expected.json")))["batched"]
    P, p_off, Q, q_off = workloads.batched()
    got = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    assert ctx.last_errors() == 0
    idx = np.array(g["sample_index"])
    assert rel_ok(got[idx], np.array(g["euclidean"]))
    want = oracle.dfd_batch(P, p_off, Q, q_off, nthreads=16)
    bad = np.flatnonzero(np.abs(got.astype(np.float64) - want) > TOL * want)
    assert bad.size == 0, f"{bad.size} pairs outside 2e-6, first {bad[:5]}"
    # end-point lower bound holds for every pair
    p0, p1 = P[p_off[:-1]].astype(np.float64), P[p_off[1:] - 1].astype(np.float64)
    q0, q1 = Q[q_off[:-1]].astype(np.float64), Q[q_off[1:] - 1].astype(np.float64)
    lb = np.maximum(np.linalg.norm(p0 - q0, axis=1), np.linalg.norm(p1 - q1, axis=1))
    assert np.all(got >= lb * (1 - TOL))
    again = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    np.testing.assert_array_equal(got, again)


def test_large_pair_full_size(ctx):
    """The single large pair (131072 x 131072 points, 3-D) in the launch the
    benchmark times: bands pipelined over every wavefront with boundary rows
    through LDS rings and global links; against the stored FP64 oracle value
    (rolling form, single thread) within 2e-6, with no device error flags."""
    say("case: large pair 131072 x 131072, 3-D")
    want = json.load(open(os.path.join(HERE, "golden", "expected.json")))["large_pair"]["euclidean"]
    p, q = workloads.large_pair()
    pd, qd = dev(p), dev(q)
    got = ctx.distance(pd, qd).item()
    assert ctx.last_errors() == 0
    info = ctx.last_launch()
    say(f"launch: {info}")
    assert info["waves"] > 1
    assert abs(got - want) <= TOL * want, (got, want)
    lb = max(np.linalg.norm(p[0].astype(np.float64) - q[0]), np.linalg.norm(p[-1].astype(np.float64) - q[-1]))
    assert got >= lb * (1 - TOL)
    # the squared form selects the same cell
    got_sq = ctx.distance(pd, qd, metric=1).item()
    assert ctx.last_errors() == 0
    assert abs(got_sq - want * want) <= 2 * TOL * want * want


def test_cross_int_workload_full_size_sampled(ctx):
    say("case: cross int workload 1024 x 1024")
    g = json.load(open(os.path.join(HERE, "golden", "expected.json")))["cross_int"]
    Qs, qo, DB, do = workloads.cross_int()
    got = ctx.cross_i32(dev(Qs), qo, dev(DB), do).cpu().numpy()
    ii, kk = np.array(g["sample_i"]), np.array(g["sample_k"])
    np.testing.assert_array_equal(got[ii, kk], np.array(g["sqeuclidean_int64"], dtype=np.int64))
    # a full row computed by the oracle now
    row = int(ii[0])
    want = oracle.dfd_cross_i32(Qs, qo, DB, do, nthreads=16, rows=[row])[0]
    np.testing.assert_array_equal(got[row], want)


def test_autotune_cache_file(ctx, tmp_path):
    """With a cache file, the autotuner writes its choice under the
    request's class, and a new context reading the file runs that shape for
    another request of the class, with the same bits."""
    from paper_2404_05708_amd import ffd
    P, p_off, Q, q_off = workloads.random_pairs(62, 300, 64, 1500, dim=2)
    path = tmp_path / "tune.json"
    say("case: autotune with a cache file")
    other = ffd.Context(0)
    try:
        other.set_tune_cache(str(path))
        t = other.autotune_batch(dev(P), p_off, dev(Q), q_off)
        entries = json.loads(path.read_text())
        assert len(entries) == 1
        (cls, e), = entries.items()
        assert cls.startswith("gfx950/") and e["rows_per_lane"] == t["rows_per_lane"]
    finally:
        other.close()
    # the same pairs in reverse order: another request of the same class
    P2, p2 = workloads.concat([P[p_off[i]:p_off[i + 1]] for i in range(299, -1, -1)])
    Q2, q2 = workloads.concat([Q[q_off[i]:q_off[i + 1]] for i in range(299, -1, -1)])
    base = ctx.batch(dev(P2), p2, dev(Q2), q2).cpu().numpy()
    fresh = ffd.Context(0)
    try:
        fresh.set_tune_cache(str(path))
        got = fresh.batch(dev(P2), p2, dev(Q2), q2).cpu().numpy()
        np.testing.assert_array_equal(got, base)
        if t["rows_per_lane"]:
            assert fresh.last_launch()["rows_per_lane"] == t["rows_per_lane"]
    finally:
        fresh.close()


def test_split_bands_bit_identical(ctx):
    """Bands split over waves (boundary rows through global links) give the
    same bits as the unsplit plan, in batch, cross and single-pair form."""
    P, p_off, Q, q_off = workloads.random_pairs(40, 60, 1, 2500, dim=2)
    say("case: split batch, 60 pairs up to 2500")
    ctx.set_split(-1.0)
    base = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    for R in (1, 2, 4, 8):
        say(f"case: split every multi-band pair, R={R}")
        ctx.set_tuning(R, 0)
        ctx.set_split(1e-9)
        try:
            got = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
            assert ctx.last_errors() == 0
        finally:
            ctx.set_split(0.0)
            ctx.set_tuning(0, 0)
        np.testing.assert_array_equal(got, base)
    want = oracle.dfd_batch(P, p_off, Q, q_off, nthreads=8)
    assert rel_ok(base, want)
    say("case: split cross int")
    Qi, qoi, Di, doi = workloads.cross_int(seed=41, nq=3, ndb=20, length=700)
    ctx.set_tuning(1, 0)
    ctx.set_split(1e-9)
    try:
        got = ctx.cross_i32(dev(Qi), qoi, dev(Di), doi).cpu().numpy()
    finally:
        ctx.set_split(0.0)
        ctx.set_tuning(0, 0)
    np.testing.assert_array_equal(got, oracle.dfd_cross_i32(Qi, qoi, Di, doi, nthreads=8))


def test_split_with_many_waves_per_simd(ctx):
    """Many split pairs mixed with unsplit ones on 3 and 4 waves per SIMD
    (small LDS shares force most multi-band pairs to split): no wave gives
    up waiting and the bits equal the unsplit plan's."""
    P, p_off, Q, q_off = workloads.random_pairs(43, 1500, 64, 2048, dim=2)
    ctx.set_split(-1.0)
    ctx.set_tuning(8, 2)
    try:
        base = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    finally:
        ctx.set_tuning(0, 0)
        ctx.set_split(0.0)
    for W, share in [(3, -1.0), (4, -1.0), (2, 0.5), (3, 0.25)]:
        say(f"case: 1500 pairs, R=8 W={W} split={share}")
        ctx.set_tuning(8, W)
        ctx.set_split(share)
        try:
            got = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
            errs = ctx.last_errors()
        finally:
            ctx.set_tuning(0, 0)
            ctx.set_split(0.0)
        assert errs == 0
        np.testing.assert_array_equal(got, base)


def test_pipelined_single_pairs(ctx):
    """A long pair as a pipeline of bands on consecutive waves: LDS rings
    inside a workgroup, global links between workgroups; partial last
    workgroups and band counts of every residue mod 4."""
    rng = np.random.default_rng(47)
    cases = [(64 * 4 * 5 + 3, 1500, 4), (64 * 2 * 6, 900, 2), (64 * 9 + 1, 700, 1), (64 * 4 * 7, 2500, 4),
             (3000, 200, 2), (64 * 2 * 2 + 5, 4000, 2)]
    for n, m, R in cases:
        say(f"case: pipelined pair n={n} m={m} R={R}")
        p = workloads.walk(rng, n, 2)
        q = workloads.walk(rng, m, 2)
        ctx.set_tuning(R, 0)
        try:
            got = ctx.distance(dev(p), dev(q)).item()
            info = ctx.last_launch()
            errs = ctx.last_errors()
        finally:
            ctx.set_tuning(0, 0)
        assert errs == 0
        assert got == oracle.dfd_f32_replica(p, q), (n, m, R, info)


def test_long_curves_force_split(ctx):
    """Column curves longer than a wave's LDS hand-off row must be split."""
    rng = np.random.default_rng(42)
    for n, m, R in [(300, 6000, 1), (700, 9000, 2), (5000, 5000, 0), (64 * 8 * 3 + 5, 3000, 8)]:
        say(f"case: long pair n={n} m={m} R={R}")
        p = workloads.walk(rng, n, 2)
        q = workloads.walk(rng, m, 2)
        ctx.set_tuning(R, 0)
        try:
            got = ctx.distance(dev(p), dev(q)).item()
            info = ctx.last_launch()
            gotb = ctx.batch(dev(p), [0, n], dev(q), [0, m]).item()
        finally:
            ctx.set_tuning(0, 0)
        say(f"  launch {info}")
        assert got == gotb
        assert got == oracle.dfd_f32_replica(p, q)
        assert rel_ok(got, oracle.dfd(p, q, 0, "rolling"))


def test_autotune_keeps_results_and_uses_the_chosen_shape(ctx):
    """The autotuner only changes launch shapes: the results stay bit for
    bit, and later calls with the same offsets run the chosen shape."""
    P, p_off, Q, q_off = workloads.random_pairs(61, 300, 64, 1500, dim=2)
    say("case: autotune batch, 300 pairs")
    base = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    t = ctx.autotune_batch(dev(P), p_off, dev(Q), q_off)
    assert t["tried"] > 0 and t["ms"] > 0
    got = ctx.batch(dev(P), p_off, dev(Q), q_off).cpu().numpy()
    np.testing.assert_array_equal(got, base)
    if t["rows_per_lane"]:
        assert ctx.last_launch()["rows_per_lane"] == t["rows_per_lane"]
    say("case: autotune cross, 6 x 300")
    Qs, qo = workloads.concat([P[p_off[i]:p_off[i + 1]] for i in range(6)])
    DB, do = workloads.concat([Q[q_off[i]:q_off[i + 1]] for i in range(300)])
    cbase = ctx.cross(dev(Qs), qo, dev(DB), do).cpu().numpy()
    ctx.autotune_cross(dev(Qs), qo, dev(DB), do)
    np.testing.assert_array_equal(ctx.cross(dev(Qs), qo, dev(DB), do).cpu().numpy(), cbase)
