"""GPU parity of the Frechet distance and DTW under the great-circle
ground distance (metric FFD_HAVERSINE) through the C ABI.

The library maps each (latitude, longitude) point to its FP64 unit vector,
sweeps Eq. (1) on squared chords and takes the central angle once per pair;
the oracle evaluates the haversine formula in every cell and sweeps the
angles.  Bar: |gpu - oracle| <= 2e-6 * oracle + 1e-12 (the float32 rounding
of the result, 2^-24 relative, plus the FP64 chord's rounding, about 1e-15
absolute before the arcsine, with margin).  Every launch shape and the
batch, cross and single-pair forms give the same bits.
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
H = oracle.HAVERSINE
HERE = os.path.dirname(os.path.abspath(__file__))


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
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def close(got, want):
    return abs(float(got) - want) <= 2e-6 * want + 1e-12


def curve(rng, n, step):
    c = workloads.geo_walk(rng, n, step)
    c[:, 1] = workloads._wrap(c[:, 1])
    return c.astype(np.float32)


@pytest.mark.parametrize("R", [0, 1, 2, 4, 8])
def test_random_shapes(ctx, R):
    rng = np.random.default_rng(720 + R)
    ctx.set_tuning(R, 0)
    try:
        for it in range(8):
            n, m = int(rng.integers(1, 700)), int(rng.integers(1, 700))
            step = float(10.0 ** rng.uniform(-5, -1))
            p, q = curve(rng, n, step), curve(rng, m, step)
            say(f"case: geo R={R} n={n} m={m} step={step:.2e}")
            got = ctx.distance(dev(p), dev(q), metric=H).item()
            want = oracle.dfd(p, q, H, "rolling")
            assert close(got, want), (R, n, m, got, want)
    finally:
        ctx.set_tuning(0, 0)


def test_batch_cross_pairs_and_split_agree(ctx):
    P, p_off, Q, q_off = workloads.geo_pairs(seed=730, npairs=150, lo=1, hi=2600)
    say("case: geo batch")
    base = ctx.batch(dev(P), p_off, dev(Q), q_off, metric=H).cpu().numpy()
    want = oracle.dfd_batch(P, p_off, Q, q_off, H, nthreads=8)
    bad = [k for k in range(len(want)) if not close(base[k], want[k])]
    assert not bad, [(k, float(base[k]), want[k]) for k in bad[:5]]
    for k in range(0, len(p_off) - 1, 25):
        p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
        assert ctx.distance(dev(p), dev(q), metric=H).item() == base[k]
    for R, share in ((2, 1e-9), (8, 1e-9), (4, 0.0)):
        say(f"case: geo batch R={R} split={share}")
        ctx.set_tuning(R, 0)
        ctx.set_split(share)
        try:
            got = ctx.batch(dev(P), p_off, dev(Q), q_off, metric=H).cpu().numpy()
            assert ctx.last_errors() == 0
        finally:
            ctx.set_split(0.0)
            ctx.set_tuning(0, 0)
        np.testing.assert_array_equal(got, base)
    Qs, qo = workloads.concat([P[p_off[k]:p_off[k + 1]] for k in range(4)])
    DB, do = workloads.concat([Q[q_off[k]:q_off[k + 1]] for k in range(30)])
    say("case: geo cross")
    cr = ctx.cross(dev(Qs), qo, dev(DB), do, metric=H).cpu().numpy()
    cw = oracle.dfd_cross(Qs, qo, DB, do, H, nthreads=8)
    assert all(close(cr[i, k], cw[i, k]) for i in range(4) for k in range(30))


def test_edge_cases(ctx):
    half = np.float32(np.pi / 2 - 1e-6)
    cases = {
        "single points": (np.array([[0.3, 1.0]]), np.array([[-0.2, -2.5]])),
        "identical": (None, None),
        "poles": (np.array([[half, 0.0], [half, 2.0], [0.0, 1.0]]), np.array([[-half, 1.0], [half, -3.0]])),
        "antipodal": (np.array([[0.5, 1.0]] * 3), np.array([[-0.5, 1.0 - np.pi]] * 2)),
        "antimeridian": (np.stack([np.zeros(50), np.linspace(3.0, 3.2, 50)], 1),
                         np.stack([np.full(40, 1e-3), np.linspace(-3.28, -3.08, 40)], 1)),
    }
    rng = np.random.default_rng(740)
    c = curve(rng, 300, 1e-3)
    for name, (p, q) in cases.items():
        if p is None:
            p = q = c
        p = np.asarray(p, np.float64)
        q = np.asarray(q, np.float64)
        for a in (p, q):
            a[:, 1] = workloads._wrap(a[:, 1])
        p, q = p.astype(np.float32), q.astype(np.float32)
        say(f"case: geo edge {name}")
        got = ctx.distance(dev(p), dev(q), metric=H).item()
        want = oracle.dfd(p, q, H, "table")
        assert close(got, want), (name, got, want)
    assert ctx.distance(dev(c), dev(c), metric=H).item() == 0.0


def test_long_pairs(ctx):
    """Long single pairs split over waves and column curves longer than the
    LDS hand-off row."""
    rng = np.random.default_rng(750)
    for n, m in [(3000, 2000), (700, 9000)]:
        p, q = curve(rng, n, 2e-3), curve(rng, m, 2e-3)
        say(f"case: geo long pair n={n} m={m}")
        got = ctx.distance(dev(p), dev(q), metric=H).item()
        assert ctx.last_errors() == 0
        assert close(got, oracle.dfd(p, q, H, "rolling"))


def dtw_close(got, want, n, m):
    # each cell's angle carries a few float32 ulps (square root and arcsine
    # of the FP64 chord), the sum is FP64, the result is rounded once
    return abs(float(got) - want) <= 2e-6 * want + 1e-12 * (n + m)


def test_dtw(ctx):
    """DTW (Appendix B) on great-circle cells: one angle per cell, summed in
    FP64, in the single-pair, batch and cross forms and across launch
    shapes."""
    P, p_off, Q, q_off = workloads.geo_pairs(seed=760, npairs=60, lo=1, hi=1500)
    say("case: geo dtw batch")
    got = ctx.dtw_batch(dev(P), p_off, dev(Q), q_off, metric=H).cpu().numpy()
    want = oracle.dtw_batch(P, p_off, Q, q_off, H, nthreads=8)
    n, m = np.diff(p_off), np.diff(q_off)
    bad = [k for k in range(60) if not dtw_close(got[k], want[k], n[k], m[k])]
    assert not bad, [(k, float(got[k]), want[k]) for k in bad[:5]]
    for k in range(0, 60, 12):
        p, q = P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]]
        assert ctx.dtw_distance(dev(p), dev(q), metric=H).item() == got[k]
    for R in (1, 2, 4, 8):
        say(f"case: geo dtw R={R}")
        ctx.set_tuning(R, 0)
        try:
            np.testing.assert_array_equal(ctx.dtw_batch(dev(P), p_off, dev(Q), q_off, metric=H).cpu().numpy(), got)
        finally:
            ctx.set_tuning(0, 0)
    Qs, qo = workloads.concat([P[p_off[k]:p_off[k + 1]] for k in range(3)])
    DB, do = workloads.concat([Q[q_off[k]:q_off[k + 1]] for k in range(20)])
    say("case: geo dtw cross")
    cr = ctx.dtw_cross(dev(Qs), qo, dev(DB), do, metric=H).cpu().numpy()
    cw = oracle.dtw_cross(Qs, qo, DB, do, H, nthreads=8)
    for i in range(3):
        for k in range(20):
            assert dtw_close(cr[i, k], cw[i, k], qo[i + 1] - qo[i], do[k + 1] - do[k])
    rng = np.random.default_rng(761)
    p, q = curve(rng, 2500, 2e-3), curve(rng, 1800, 2e-3)
    say("case: geo dtw long pair")
    assert dtw_close(ctx.dtw_distance(dev(p), dev(q), metric=H).item(), oracle.dtw(p, q, H), 2500, 1800)
    assert ctx.last_errors() == 0


def test_full_workload_sampled(ctx):
    """The 4096-pair sphere workload in the launch configuration bench.py
    times, checked on the pairs the stored values cover."""
    g = json.load(open(os.path.join(HERE, "golden", "expected.json")))["batched_haversine"]
    P, p_off, Q, q_off = workloads.geo_pairs()
    say("case: geo full workload")
    got = ctx.batch(dev(P), p_off, dev(Q), q_off, metric=H).cpu().numpy()
    assert ctx.last_errors() == 0
    for k, want in zip(g["sample_index"], g["haversine"]):
        assert close(got[k], want), (k, float(got[k]), want)


def test_refused_forms(ctx):
    from paper_2404_05708_amd import ffd
    p = dev(np.zeros((4, 3), np.float32))
    with pytest.raises(ffd.FFDError) as e:
        ctx.distance(p, p, metric=H)
    assert e.value.status == ffd.FFD_E_INVALID
    pi = torch.zeros((4, 2), dtype=torch.int32, device="cuda:0")
    with pytest.raises(ffd.FFDError) as e:
        ctx.distance_i32(pi, pi, metric=H)
    assert e.value.status == ffd.FFD_E_UNSUPPORTED
