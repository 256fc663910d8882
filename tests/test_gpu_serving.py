"""GPU serving: queries against a resident database with continuous batching.

Each query's distances to every database curve must be the same, bit for
bit, when the query runs alone and when it runs mixed with others admitted
into the same or overlapping launches; they must equal ffd_cross on the
same inputs bit for bit, and the FP64 oracle within a relative 2e-6.
"""
import sys
import threading

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
def served(gpu):
    from paper_2404_05708_amd import ffd
    ctx = ffd.Context(0)
    # a smaller database with the serving length law, plus long curves so
    # that long queries need boundary rows that do not fit LDS
    DB, dbo = workloads.serving_db(seed=51, count=1500)
    rng = np.random.default_rng(52)
    extra = [workloads.walk(rng, L, 2) for L in (3000, 5000, 8192)]
    parts = [DB[dbo[k]:dbo[k + 1]] for k in range(len(dbo) - 1)] + extra
    DB, dbo = workloads.concat(parts)
    DBd = torch.from_numpy(DB).to("cuda:0")
    db = ffd.Database(ctx, DBd, dbo)
    srv = ffd.Server(db, max_slots=8, max_query=8192)
    yield ffd, ctx, DB, dbo, DBd, srv
    srv.close()
    db.close()
    torch.cuda.synchronize()
    ctx.close()


def queries():
    qs = workloads.serving_queries(seed=53, count=10)
    rng = np.random.default_rng(54)
    qs.append(workloads.walk(rng, 2600, 2))   # several bands, long database curves
    qs.append(workloads.walk(rng, 40, 2))
    return qs


def test_alone_equals_mix_equals_cross(served):
    ffd, ctx, DB, dbo, DBd, srv = served
    qs = queries()
    say(f"case: serving, {len(qs)} queries alone, db {len(dbo) - 1} curves")
    alone = []
    for q in qs:
        alone.append(srv.wait(srv.submit(q)).copy())
    say("case: serving, all queries at once")
    tickets = [srv.submit(q) for q in qs]
    mix = [srv.wait(t).copy() for t in tickets]
    for a, b in zip(alone, mix):
        np.testing.assert_array_equal(a, b)
    say("case: serving, mixed from two threads")
    res = {}

    def client(idx):
        for i in idx:
            res[i] = srv.wait(srv.submit(qs[i])).copy()
    th = [threading.Thread(target=client, args=(range(j, len(qs), 2),)) for j in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i in range(len(qs)):
        np.testing.assert_array_equal(res[i], alone[i])
    say("case: serving vs ffd_cross")
    Qs, qo = workloads.concat(qs)
    cross = ctx.cross(torch.from_numpy(Qs).to("cuda:0"), qo, DBd, dbo).cpu().numpy()
    for i in range(len(qs)):
        np.testing.assert_array_equal(alone[i], cross[i])
    say("case: serving vs oracle")
    pick = [0, len(qs) - 2, len(qs) - 1]
    sq, so = workloads.concat([qs[i] for i in pick])
    want = oracle.dfd_cross(sq, so, DB, dbo, oracle.EUCLIDEAN, nthreads=8)
    for r, i in enumerate(pick):
        got = alone[i].astype(np.float64)
        assert np.all(np.abs(got - want[r]) <= TOL * np.abs(want[r]))


def test_rows_per_lane_shapes(served):
    """Query lengths for which the server picks each of 1 ... 8 rows per
    lane (including 3, 5, 6 and 7, and those over several bands): alone, in
    a mix, against ffd_cross bit for bit and the oracle within 2e-6."""
    ffd, ctx, DB, dbo, DBd, srv = served
    rng = np.random.default_rng(55)
    lens = [40, 100, 150, 220, 300, 360, 420, 480, 600, 700, 1200, 2600]
    qs = [workloads.walk(rng, L, 2) for L in lens]
    say(f"case: serving shapes, lengths {lens}")
    srv.reset_stats()
    alone = [srv.wait(srv.submit(q)).copy() for q in qs]
    by_rows = srv.stats()["launches_by_rows"]
    say(f"launches by rows per lane: {by_rows}")
    # a query over more bands than one item holds takes several launches
    assert sum(by_rows) >= len(qs) and all(by_rows[r - 1] > 0 for r in (3, 5, 6, 7)), by_rows
    tickets = [srv.submit(q) for q in qs]
    mix = [srv.wait(t).copy() for t in tickets]
    Qs, qo = workloads.concat(qs)
    cross = ctx.cross(torch.from_numpy(Qs).to("cuda:0"), qo, DBd, dbo).cpu().numpy()
    for i in range(len(qs)):
        np.testing.assert_array_equal(alone[i], mix[i])
        np.testing.assert_array_equal(alone[i], cross[i])
    pick = [lens.index(L) for L in (150, 300, 600, 1200)]
    sq, so = workloads.concat([qs[i] for i in pick])
    want = oracle.dfd_cross(sq, so, DB, dbo, oracle.EUCLIDEAN, nthreads=8)
    for r, i in enumerate(pick):
        got = alone[i].astype(np.float64)
        assert np.all(np.abs(got - want[r]) <= TOL * np.abs(want[r])), lens[i]


def test_metrics_and_stats(served):
    ffd, ctx, DB, dbo, DBd, srv = served
    q = queries()[3]
    srv.reset_stats()
    e = srv.wait(srv.submit(q, ffd.FFD_EUCLIDEAN)).astype(np.float64)
    s = srv.wait(srv.submit(q, ffd.FFD_SQEUCLIDEAN)).astype(np.float64)
    assert np.all(np.abs(s - e * e) <= 4 * TOL * s + 1e-30)
    st = srv.stats()
    assert st["completed"] == 2 and st["failed"] == 0
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]


def test_poll_and_errors(served):
    ffd, ctx, DB, dbo, DBd, srv = served
    q = queries()[0]
    t = srv.submit(q)
    while srv.poll(t) is None:
        pass
    with pytest.raises(ffd.FFDError):
        srv.poll(t)  # collected
    with pytest.raises(ffd.FFDError):
        srv.submit(np.zeros((9000, 2), dtype=np.float32))  # longer than max_query
    with pytest.raises(ffd.FFDError):
        srv.submit(np.zeros((0, 2), dtype=np.float32))
    with pytest.raises(ffd.FFDError) as ei:
        srv.submit(q, ffd.FFD_MANHATTAN)  # serving takes the Euclidean metrics only
    assert ei.value.status == ffd.FFD_E_UNSUPPORTED


def test_long_queries_in_items(served):
    """Queries of 5000 to 8192 points are swept a few bands per launch, their
    boundary rows kept in the request's buffers between launches, while
    short queries run in the launches between; more long queries than
    buffer pairs wait for a pair.  Every result equals the query alone and
    ffd_cross bit for bit."""
    ffd, ctx, DB, dbo, DBd, srv = served
    rng = np.random.default_rng(56)
    longs = [workloads.walk(rng, L, 2) for L in (8192, 5000, 7000, 6000, 8192, 5500, 6500, 7500, 8000, 5200)]
    shorts = [workloads.walk(rng, int(L), 2) for L in rng.integers(32, 400, size=30)]
    say(f"case: serving, {len(longs)} long queries (more than the 8 buffer pairs) and {len(shorts)} short ones")
    alone_long = [srv.wait(srv.submit(q)).copy() for q in longs[:2]]
    srv.reset_stats()
    order = []
    tickets = []
    for i in range(max(len(longs), len(shorts))):
        for kind, qs in (("L", longs), ("S", shorts)):
            if i < len(qs):
                tickets.append((kind, i, srv.submit(qs[i])))
    got = {(k, i): srv.wait(t).copy() for k, i, t in tickets}
    st = srv.stats()
    say(f"stats: {st}")
    assert st["completed"] == len(longs) + len(shorts) and st["failed"] == 0
    assert sum(st["launches_by_rows"]) > len(tickets) // srv_items_per_launch(st)
    for i in range(2):
        np.testing.assert_array_equal(got[("L", i)], alone_long[i])
    allq = longs + shorts
    Qs, qo = workloads.concat(allq)
    cross = ctx.cross(torch.from_numpy(Qs).to("cuda:0"), qo, DBd, dbo).cpu().numpy()
    for i in range(len(longs)):
        np.testing.assert_array_equal(got[("L", i)], cross[i])
    for i in range(len(shorts)):
        np.testing.assert_array_equal(got[("S", i)], cross[len(longs) + i])
    want = oracle.dfd_cross(longs[1], [0, len(longs[1])], DB, dbo, oracle.EUCLIDEAN, nthreads=16)[0]
    assert np.all(np.abs(got[("L", 1)].astype(np.float64) - want) <= TOL * np.abs(want))


def test_cancel_and_deadline(served):
    """A request canceled while it waits, or between two of its launches,
    reports FFD_E_CANCELED and its results array is never written; the
    watchdog drops a long query whose next launch would come after its
    deadline (FFD_E_EXPIRED); requests around them complete with their usual
    bits."""
    ffd, ctx, DB, dbo, DBd, srv = served
    rng = np.random.default_rng(57)
    longs = [workloads.walk(rng, 8192, 2) for _ in range(10)]
    short = workloads.walk(rng, 300, 2)
    alone_short = srv.wait(srv.submit(short)).copy()
    srv.reset_stats()
    ndb = len(dbo) - 1
    sentinel = np.float32(-7.0)
    outs = [np.full(ndb, sentinel, dtype=np.float32) for _ in longs]
    # 10 queries that each need a boundary-row buffer pair; the server has 8
    say("case: serving, cancel two waiting long queries and one running")
    tickets = [srv.submit(q, out=o) for q, o in zip(longs, outs)]
    for t in (tickets[-1], tickets[-2], tickets[0]):
        srv.cancel(t)
    for j in (-1, -2):
        with pytest.raises(ffd.FFDError) as ei:
            srv.wait(tickets[j])
        assert ei.value.status == ffd.FFD_E_CANCELED
        assert np.all(outs[j] == sentinel)
    try:
        srv.wait(tickets[0])
        first_canceled = False
    except ffd.FFDError as e:
        assert e.status == ffd.FFD_E_CANCELED
        assert np.all(outs[0] == sentinel)
        first_canceled = True
    done = [srv.wait(t).copy() for t in tickets[1:-2]]
    Qs, qo = workloads.concat(longs[1:3])
    cross = ctx.cross(torch.from_numpy(Qs).to("cuda:0"), qo, DBd, dbo).cpu().numpy()
    np.testing.assert_array_equal(done[0], cross[0])
    np.testing.assert_array_equal(done[1], cross[1])
    st = srv.stats()
    say(f"stats after cancel: {st}")
    assert st["canceled"] == 2 + int(first_canceled) and st["completed"] == 7 + int(not first_canceled)
    say("case: serving, deadline of 100 us on a long query")
    srv.set_deadline(100)
    try:
        out = np.full(ndb, sentinel, dtype=np.float32)
        t = srv.submit(longs[3], out=out)
        with pytest.raises(ffd.FFDError) as ei:
            srv.wait(t)
        assert ei.value.status == ffd.FFD_E_EXPIRED
        assert np.all(out == sentinel)
    finally:
        srv.set_deadline(0)
    np.testing.assert_array_equal(srv.wait(srv.submit(short)), alone_short)
    st = srv.stats()
    assert st["expired"] == 1
    with pytest.raises(ffd.FFDError):
        srv.cancel(123456789)  # unknown ticket
    with pytest.raises(ffd.FFDError):
        srv.set_deadline(-1)


def srv_items_per_launch(st):
    return max(1, st["requests_per_launch"])
