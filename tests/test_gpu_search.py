"""GPU parity of the decider and the k-nearest-neighbour search (early
abandoning) through the C ABI.

Expected values come from the oracle's float32 replica, which the GPU's
squared-cell Frechet path equals bit for bit (one square root per pair, in
FP64, rounded once): the decider must give exactly where(delta <= eps,
delta, +inf) and the search exactly the k smallest (delta, index) pairs.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


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


def replica(P, p_off, Q, q_off, metric):
    n = len(p_off) - 1
    out = np.empty(n, dtype=np.float32)
    for k in range(n):
        out[k] = oracle.dfd_f32_replica(P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]], metric)
    return out


@pytest.mark.parametrize("metric", [0, 1])
def test_decider_matches_replica(ctx, metric):
    # lengths from 1 to 1300: single bands and up to three bands at R = 8,
    # column curves longer and shorter than a group
    P, p_off, Q, q_off = workloads.random_pairs(820 + metric, 90, 1, 1300, dim=2)
    want = replica(P, p_off, Q, q_off, metric)
    base = ctx.batch(dev(P), p_off, dev(Q), q_off, metric=metric).cpu().numpy()
    np.testing.assert_array_equal(base, want)
    for q in (0.0, 0.1, 0.5, 0.9, 1.0):
        eps = float(np.quantile(want, q))
        say(f"case: decider metric={metric} eps=quantile {q}")
        got = ctx.decide_batch(dev(P), p_off, dev(Q), q_off, eps, metric=metric).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.decide(want, np.float32(eps)))
    for eps in (np.inf, -1.0, 0.0):
        say(f"case: decider metric={metric} eps={eps}")
        got = ctx.decide_batch(dev(P), p_off, dev(Q), q_off, eps, metric=metric).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.decide(want, np.float32(eps)))


def test_decider_close_pairs_and_dims(ctx):
    """Pairs whose distances sit just around the threshold, near copies of
    each other (early abandoning is rare there), 1-D and 3-D curves."""
    P, p_off, Q, q_off = workloads.batched(seed=830, npairs=60, lo=20, hi=900, dim=2)
    want = replica(P, p_off, Q, q_off, 0)
    for eps in np.sort(want)[::7]:
        for e in (np.nextafter(eps, np.float32(0)), eps, np.nextafter(eps, np.float32(np.inf))):
            got = ctx.decide_batch(dev(P), p_off, dev(Q), q_off, float(e)).cpu().numpy()
            np.testing.assert_array_equal(got, oracle.decide(want, e))
    for D in (1, 3):
        P, p_off, Q, q_off = workloads.random_pairs(831 + D, 40, 1, 700, dim=D)
        want = replica(P, p_off, Q, q_off, 0)
        eps = float(np.median(want))
        say(f"case: decider D={D}")
        got = ctx.decide_batch(dev(P), p_off, dev(Q), q_off, eps).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.decide(want, np.float32(eps)))


@pytest.mark.parametrize("k", [1, 5, 40, 400])
def test_knn_matches_replica(ctx, k):
    DB, db_off = workloads.serving_db(seed=840, count=300, lo=8, hi=1500)
    queries = workloads.serving_queries(seed=841, count=4, lo=8, hi=900)
    for i in range(4):
        q = queries[i]
        say(f"case: knn k={k} query {i} n={len(q)}")
        vals = np.array([oracle.dfd_f32_replica(q, DB[db_off[c]:db_off[c + 1]], 0) for c in range(300)],
                        dtype=np.float32)
        want_i, want_d = oracle.knn(vals, k)
        gi, gd = ctx.knn(dev(q), dev(DB), db_off, k)
        np.testing.assert_array_equal(gd.cpu().numpy(), want_d)
        np.testing.assert_array_equal(gi.cpu().numpy(), want_i)
        info = ctx.last_search()
        assert info["exact"] + info["bounded"] <= 300 and info["rejected"] <= info["bounded"]


@pytest.mark.parametrize("k,metric", [(1, 0), (10, 0), (40, 1), (400, 0)])
def test_knn_batch_matches_replica(ctx, k, metric):
    """Several queries in one ffd_knn_batch call (lengths spanning one to
    several bands, so the per-pair row mapping and the per-query thresholds
    are both exercised): each query's k nearest equal the replica's, and
    equal ffd_knn of that query alone."""
    DB, db_off = workloads.serving_db(seed=860 + k, count=300, lo=8, hi=1500)
    queries = workloads.serving_queries(seed=861 + k, count=7, lo=8, hi=1400)
    Qs, q_off = workloads.concat(queries)
    say(f"case: knn batch k={k} metric={metric} nq=7 lengths={[len(q) for q in queries]}")
    gi, gd = ctx.knn_batch(dev(Qs), q_off, dev(DB), db_off, k, metric=metric)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    assert gi.shape == (7, k) and gd.shape == (7, k)
    for i, q in enumerate(queries):
        vals = np.array([oracle.dfd_f32_replica(q, DB[db_off[c]:db_off[c + 1]], metric) for c in range(300)],
                        dtype=np.float32)
        want_i, want_d = oracle.knn(vals, k)
        np.testing.assert_array_equal(gd[i], want_d)
        np.testing.assert_array_equal(gi[i], want_i)
        si, sd = ctx.knn(dev(q), dev(DB), db_off, k, metric=metric)
        np.testing.assert_array_equal(si.cpu().numpy(), gi[i])
        np.testing.assert_array_equal(sd.cpu().numpy(), gd[i])


def test_knn_prunes_and_squared_metric(ctx):
    """A database of noisy copies of a few templates: the nearest curves are
    the query's own template, most others are bounded out or dropped."""
    rng = np.random.default_rng(850)
    templates = [workloads.walk(rng, int(rng.integers(200, 700)), 2) for _ in range(10)]
    curves = []
    for c in range(600):
        t = templates[c % 10]
        curves.append((t + 0.2 * rng.standard_normal(t.shape)).astype(np.float32))
    DB, db_off = workloads.concat(curves)
    q = (templates[3] + 0.2 * rng.standard_normal(templates[3].shape)).astype(np.float32)
    vals = np.array([oracle.dfd_f32_replica(q, DB[db_off[c]:db_off[c + 1]], 1) for c in range(600)],
                    dtype=np.float32)
    want_i, want_d = oracle.knn(vals, 10)
    gi, gd = ctx.knn(dev(q), dev(DB), db_off, 10, metric=1)
    np.testing.assert_array_equal(gd.cpu().numpy(), want_d)
    np.testing.assert_array_equal(gi.cpu().numpy(), want_i)
    info = ctx.last_search()
    say(f"search counts: {info}")
    assert info["exact"] + info["bounded"] < 600


def test_refused_forms(ctx):
    from paper_2404_05708_amd import ffd
    p = dev(np.zeros((4, 2), np.float32))
    with pytest.raises(ffd.FFDError) as e:
        ctx.decide_batch(p, [0, 4], p, [0, 4], 1.0, metric=ffd.FFD_MANHATTAN)
    assert e.value.status == ffd.FFD_E_UNSUPPORTED
    with pytest.raises(ffd.FFDError) as e:
        ctx.decide_batch(p, [0, 4], p, [0, 4], float("nan"))
    assert e.value.status == ffd.FFD_E_INVALID
    with pytest.raises(ffd.FFDError) as e:
        ctx.knn(p, p, [0, 2, 4], 0)
    assert e.value.status == ffd.FFD_E_INVALID
