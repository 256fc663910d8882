"""Launch plans replayed on the CPU by the schedule simulator (no GPU).

A planning-only context (256 CUs, 160 KB of LDS per CU) builds the plans
the library would launch for the benchmark workloads, for forced band
splitting, other launch shapes, long curves whose boundary rows do not fit
LDS, cross requests, single long pairs (the LDS-ring pipeline) and the DTW,
Manhattan, Chebyshev, Levenshtein and great-circle kernels; tests/plan_sim.py checks coverage, output indices,
hand-off adjacency, link and ring lags (deadlock freedom) and buffer bounds.
"""
import numpy as np
import pytest

from paper_2404_05708_amd import ffd
import plan_sim
import workloads


@pytest.fixture
def planner():
    h = ffd.ffd_create_planner(256, 160 * 1024)
    yield h
    ffd.ffd_destroy(h)


def batch_case(h, p_off, q_off, dim=2, **kw):
    sm, jobs, wj = ffd.ffd_plan_describe(h, ffd.FFD_OP_BATCH, p_off, q_off, dim, **kw)
    plan_sim.check(sm, jobs, wj, (np.asarray(p_off), np.asarray(q_off)), range(len(p_off) - 1))
    return sm


def test_batched_workload_plan(planner):
    P, p_off, Q, q_off = workloads.batched()
    sm = batch_case(planner, p_off, q_off)
    assert sm["rows_per_lane"] == 8 and sm["waves"] == 2048 and sm["cooperative"] == 1


@pytest.mark.parametrize("R,W", [(1, 0), (2, 0), (4, 0), (8, 0), (8, 3), (4, 4)])
def test_forced_split_and_launch_shapes(planner, R, W):
    P, p_off, Q, q_off = workloads.random_pairs(400 + R, 300, 1, 2500, dim=2)
    ffd.ffd_set_tuning(planner, R, W)
    try:
        batch_case(planner, p_off, q_off)
        ffd.ffd_set_split(planner, 1e-9)
        sm = batch_case(planner, p_off, q_off)
        assert sm["flags"] > 0
    finally:
        ffd.ffd_set_split(planner, 0.0)
        ffd.ffd_set_tuning(planner, 0, 0)


def test_long_curves_chain_through_links(planner):
    # column curves longer than a wave's LDS hand-off row: bands chain
    # through global links, split or in place on one wave
    P, p_off, Q, q_off = workloads.random_pairs(410, 120, 1, 9000, dim=2)
    sm = batch_case(planner, p_off, q_off)
    assert sm["flags"] > 0
    ffd.ffd_set_split(planner, -1.0)
    try:
        batch_case(planner, p_off, q_off)
    finally:
        ffd.ffd_set_split(planner, 0.0)


def test_cross_plans(planner):
    Qs, qo, DB, do = workloads.cross_int()
    sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_CROSS, qo, do, 2, exact=True, metric=1)
    nq, ndb = len(qo) - 1, len(do) - 1
    plan_sim.check(sm, jobs, wj, (qo, do), range(nq * ndb))
    rng = np.random.default_rng(411)
    qo2 = np.concatenate([[0], np.cumsum(rng.integers(1, 3000, size=20))]).astype(np.int64)
    do2 = np.concatenate([[0], np.cumsum(rng.integers(1, 9000, size=60))]).astype(np.int64)
    sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_CROSS, qo2, do2, 3)
    plan_sim.check(sm, jobs, wj, (qo2, do2), range(20 * 60))


@pytest.mark.parametrize("n,m,dim", [(131072, 131072, 3), (512, 384, 2), (5000, 5000, 2), (64 * 4 * 7, 2500, 2)])
def test_single_pairs(planner, n, m, dim):
    """Long single Frechet pairs go to the pipelined kernel (no job table):
    one band of 64 R rows per wave, four waves per workgroup, one link row
    per workgroup boundary; the job-table planner's own pair plans (R = 1,
    where the pipelined kernel does not run) still pass the simulator."""
    sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_PAIR, [0, n], [0, m], dim)
    assert sm["pipelined"] == 1 and sm["jobs"] == 0
    R = sm["rows_per_lane"]
    shapes = []  # (bands, link values) with either curve holding the rows
    for rows, cols in ((n, m), (m, n)):
        bands = -(-rows // (64 * R))
        shapes.append((bands, ((bands - 1) // 4) * (-(-cols // 64) * 64)))
    assert any(sm["link_elems"] == le and (sm["waves"] >= nb or sm["waves"] == 1024) for nb, le in shapes)
    if n == 131072:
        assert R == 2 and sm["waves"] == 1024
    ffd.ffd_set_tuning(planner, 1, 0)
    try:
        sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_PAIR, [0, n], [0, m], dim)
    finally:
        ffd.ffd_set_tuning(planner, 0, 0)
    assert sm["pipelined"] == 0
    plan_sim.check(sm, jobs, wj, (np.array([0, n]), np.array([0, m])), [0])


def test_forced_pipeline(planner):
    """waves_per_simd = -1 puts a pair on the pipelined kernel whenever that
    kernel can run it, in the orientation of least modelled time; one that
    it cannot run (a single band) stays on the job-table plan."""
    ffd.ffd_set_tuning(planner, 2, -1)
    try:
        sm, jobs, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_PAIR, [0, 5000], [0, 3], 2)
        assert sm["pipelined"] == 1 and sm["rows_per_lane"] == 2 and sm["jobs"] == 0
        bands = -(-5000 // 128)
        assert sm["link_elems"] == ((bands - 1) // 4) * 64
        sm, _, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_PAIR, [0, 300], [0, 20000], 2)
        assert sm["pipelined"] == 1 and sm["link_elems"] == ((-(-20000 // 128) - 1) // 4) * 320
        sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_PAIR, [0, 100], [0, 90], 2)
        assert sm["pipelined"] == 0
        plan_sim.check(sm, jobs, wj, (np.array([0, 100]), np.array([0, 90])), [0])
    finally:
        ffd.ffd_set_tuning(planner, 0, 0)


@pytest.mark.parametrize("dtw,metric,lev", [(True, 1, False), (True, 0, False), (False, 2, False),
                                            (True, 3, False), (False, 1, True), (False, 4, False),
                                            (True, 4, False)])
def test_other_kernels(planner, dtw, metric, lev):
    P, p_off, Q, q_off = workloads.random_pairs(412, 200, 1, 6000, dim=2)
    sm = batch_case(planner, p_off, q_off, dtw=dtw, metric=metric, exact=lev, levenshtein=lev)
    assert sm["rings"] == 0
    smp, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_PAIR, [0, 40000], [0, 30000], 2, dtw=dtw,
                                          metric=metric, exact=lev, levenshtein=lev)
    plan_sim.check(smp, jobs, wj, (np.array([0, 40000]), np.array([0, 30000])), [0])
    assert smp["rings"] == 0


def test_simulator_catches_a_broken_plan(planner):
    """Planted mistakes in a copy of a real plan (CPU only): a link consumer
    moved closer to its producer, a dropped band, a duplicated output."""
    P, p_off, Q, q_off = workloads.random_pairs(413, 200, 1, 2500, dim=2)
    ffd.ffd_set_tuning(planner, 2, 0)
    ffd.ffd_set_split(planner, 1e-9)
    try:
        sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, p_off, q_off, 2)
    finally:
        ffd.ffd_set_split(planner, 0.0)
        ffd.ffd_set_tuning(planner, 0, 0)
    offs = (np.asarray(p_off), np.asarray(q_off))
    plan_sim.check(sm, jobs, wj, offs, range(len(p_off) - 1))
    # 1: shorten the idle padding in front of a link consumer
    idle = np.nonzero((jobs["row_sel"] == 2) & (jobs["col_count"] >= 16))[0]
    assert len(idle) > 0
    bad = jobs.copy()
    bad["col_count"][idle[0]] -= 16
    sm2 = dict(sm)
    tasks, ends = plan_sim.replay(sm2, bad, wj, offs)
    sm2["stream_steps"] = max(ends)
    with pytest.raises(AssertionError):
        plan_sim.check(sm2, bad, wj, offs, range(len(p_off) - 1))
    # 2: a job that drops its last band
    multi = np.nonzero((jobs["row_sel"] != 2) & (jobs["band_count"] > 1))[0]
    if len(multi):
        bad = jobs.copy()
        bad["band_count"][multi[0]] -= 1
        with pytest.raises(AssertionError):
            plan_sim.check(sm, bad, wj, offs, range(len(p_off) - 1))
    # 3: two pairs writing one output
    tasks, _ = plan_sim.replay(sm, jobs, wj, offs)
    writers = sorted({t["job"] for t in tasks if t["out"] is not None})
    bad = jobs.copy()
    bad["out_base"][writers[1]] = bad["out_base"][writers[0]]
    with pytest.raises(AssertionError):
        plan_sim.check(sm, bad, wj, offs, range(len(p_off) - 1))


@pytest.mark.parametrize("dim,R", [(5, 2), (8, 2), (9, 1), (16, 1)])
def test_wide_dimensions(planner, dim, R):
    """Curves of 5 to 16 coordinates run on the kernels of 8 (R = 2) or 16
    (R = 1) coordinates: batch, cross and single-pair plans take that R, pass
    the simulator, and a long pair stays on the job-table plan (the pipelined
    kernel has no wide form), also when the pipeline is asked for."""
    P, p_off, Q, q_off = workloads.random_pairs(300, 300, 1, 2500, dim=2)
    sm = batch_case(planner, p_off, q_off, dim=dim)
    assert sm["rows_per_lane"] == R
    sm = batch_case(planner, p_off, q_off, dim=dim, exact=True, metric=ffd.FFD_SQEUCLIDEAN)
    assert sm["rows_per_lane"] == R
    sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_CROSS, p_off[:21], q_off, dim, dtw=True)
    assert sm["rows_per_lane"] == R
    plan_sim.check(sm, jobs, wj, (np.asarray(p_off[:21]), np.asarray(q_off)), range(20 * 300))
    for w in (0, -1):
        ffd.ffd_set_tuning(planner, 0, w)
        try:
            sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_PAIR, [0, 20000], [0, 20000], dim)
        finally:
            ffd.ffd_set_tuning(planner, 0, 0)
        assert sm["pipelined"] == 0 and sm["rows_per_lane"] == R
        plan_sim.check(sm, jobs, wj, (np.array([0, 20000]), np.array([0, 20000])), [0])
    # a forced rows-per-lane other than the wide kernel's is refused
    ffd.ffd_set_tuning(planner, 4 if R != 4 else 8, 0)
    try:
        with pytest.raises(ffd.FFDError) as e:
            ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, p_off, q_off, dim)
        assert e.value.status == ffd.FFD_E_UNSUPPORTED
    finally:
        ffd.ffd_set_tuning(planner, 0, 0)


def test_short_pairs_per_lane(planner):
    """A batch whose pairs all have a curve of at most 64 points (32 for
    3-D and 4-D, half that for the exact path) runs one pair per lane when
    the model prefers it (the Frechet distance and DTW on squared Euclidean,
    Manhattan or Chebyshev cells, DTW also on Euclidean cells, Levenshtein);
    a long pair among them goes to the job-table plan alone; a forced launch
    shape, the great-circle distance or a split setting keeps the job-table
    plan for all."""
    def offsets(seed, count, lo, hi):
        rng = np.random.default_rng(seed)
        a = np.concatenate([[0], np.cumsum(rng.integers(lo, hi + 1, size=count))]).astype(np.int64)
        b = np.concatenate([[0], np.cumsum(rng.integers(lo, hi + 1, size=count))]).astype(np.int64)
        return a, b

    # a few thousand pairs: a lane sweeps its whole pair alone, so the
    # streaming kernel (64 rows of a pair in parallel) finishes first
    p_off, q_off = offsets(69, 5000, 1, 64)
    assert batch_case(planner, p_off, q_off)["per_lane"] == 0
    # many pairs: one per lane
    p_off, q_off = offsets(70, 200000, 1, 64)
    sm, jobs, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, p_off, q_off, 2)
    assert sm["per_lane"] == 1 and sm["jobs"] == 0 and sm["rows_per_lane"] == 0
    lens = np.maximum(np.diff(p_off), np.diff(q_off))
    assert sm["stream_steps"] == lens.max()
    # classes of column count, multiples of 8: waves = pairs per class / 64, rounded up
    short = np.minimum(np.diff(p_off), np.diff(q_off))
    per = np.bincount((short - 1) // 8, minlength=8)
    assert sm["waves"] == sum(-(-int(c) // 64) for c in per)
    # Levenshtein: the column curve is the one leaving less padded work
    # (rows two at a time, columns to a multiple of 8), the shorter on a tie
    sm = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, p_off, q_off, 1, exact=True, levenshtein=True)[0]
    n, m = np.diff(p_off), np.diff(q_off)
    padded = lambda r, c: (r + 1) // 2 * 2 * ((c + 7) // 8 * 8)
    turn, keep = padded(m, n), padded(n, m)
    swap = (turn < keep) | ((turn == keep) & (n < m))
    cols, rows = np.where(swap, n, m), np.where(swap, m, n)
    assert np.sum(padded(rows, cols)) < np.sum(padded(np.maximum(n, m), np.minimum(n, m)))
    assert sm["per_lane"] == 1 and sm["stream_steps"] == rows.max()
    assert sm["waves"] == sum(-(-int(c) // 64) for c in np.bincount((cols - 1) // 8, minlength=8))
    # one long pair as well: it alone goes to the streaming kernel
    p2 = np.concatenate([p_off, [p_off[-1] + 500]])
    q2 = np.concatenate([q_off, [q_off[-1] + 500]])
    sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, p2, q2, 2)
    assert sm["per_lane"] == 1 and sm["jobs"] > 0
    plan_sim.check(sm, jobs, wj, (p2, q2), [len(p2) - 2])
    # 3-D curves hold at most 32 columns per lane, the exact path 32 (2-D):
    # the pairs with a curve of at most 32 points per lane, the rest on the
    # job-table plan
    sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, p_off, q_off, 3)
    assert sm["per_lane"] == 1 and sm["jobs"] > 0
    short = np.minimum(np.diff(p_off), np.diff(q_off))
    plan_sim.check(sm, jobs, wj, (p_off, q_off), np.nonzero(short > 32)[0])
    pb, qb = offsets(71, 200000, 1, 32)
    sm, _, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, pb, qb, 3)
    assert sm["per_lane"] == 1
    sm, _, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, pb, qb, 2, exact=True, metric=ffd.FFD_SQEUCLIDEAN)
    assert sm["per_lane"] == 1
    for metric in (ffd.FFD_MANHATTAN, ffd.FFD_CHEBYSHEV):  # the Frechet distance on other cells
        sm, _, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, pb, qb, 2, metric=metric)
        assert sm["per_lane"] == 1
    sm, _, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, pb, qb, 2, dtw=True)
    assert sm["per_lane"] == 1  # DTW too
    sm, _, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, pb, qb, 1, levenshtein=True, exact=True)
    assert sm["per_lane"] == 1  # Levenshtein too
    assert batch_case(planner, pb, qb, dim=2, metric=ffd.FFD_HAVERSINE)["per_lane"] == 0
    ffd.ffd_set_tuning(planner, 1, 0)
    try:
        assert batch_case(planner, pb, qb, dim=2)["per_lane"] == 0
    finally:
        ffd.ffd_set_tuning(planner, 0, 0)
    ffd.ffd_set_split(planner, 1.5)
    try:
        assert batch_case(planner, pb, qb, dim=2)["per_lane"] == 0
    finally:
        ffd.ffd_set_split(planner, 0.0)


def test_short_and_long_pairs(planner):
    """A batch of many short pairs and some long ones: the short ones run one
    per lane, the rest on the streaming kernel's job-table plan (which the
    simulator checks for exactly the long pairs' outputs); a batch of few
    short pairs keeps one job-table plan for all."""
    rng = np.random.default_rng(72)
    n = np.concatenate([rng.integers(1, 65, size=200000), rng.integers(500, 2001, size=3000)])
    m = np.concatenate([rng.integers(1, 65, size=200000), rng.integers(500, 2001, size=3000)])
    perm = rng.permutation(len(n))
    n, m = n[perm], m[perm]
    p_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    q_off = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_BATCH, p_off, q_off, 2)
    assert sm["per_lane"] == 1 and sm["jobs"] > 0
    long_pairs = np.nonzero(np.minimum(n, m) > 64)[0]
    assert len(long_pairs) == 3000
    plan_sim.check(sm, jobs, wj, (p_off, q_off), long_pairs)
    few = np.concatenate([[0], np.cumsum(np.concatenate([rng.integers(1, 65, size=300), [1500]]))]).astype(np.int64)
    assert batch_case(planner, few, few)["per_lane"] == 0


def test_short_cross_per_lane(planner):
    """Queries x database with every curve short: one (query, curve) pair
    per lane when the model prefers it; one long query keeps the job-table
    plan (a cross request is not split)."""
    rng = np.random.default_rng(73)
    qo = np.concatenate([[0], np.cumsum(rng.integers(2, 49, size=500))]).astype(np.int64)
    do = np.concatenate([[0], np.cumsum(rng.integers(2, 49, size=400))]).astype(np.int64)
    sm, jobs, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_CROSS, qo, do, 2)
    assert sm["per_lane"] == 1 and sm["jobs"] == 0
    sm, _, _ = ffd.ffd_plan_describe(planner, ffd.FFD_OP_CROSS, qo, do, 2, dtw=True)
    assert sm["per_lane"] == 1
    q2 = np.concatenate([qo, [qo[-1] + 3000]])
    d2 = np.concatenate([do, [do[-1] + 3000]])
    sm, jobs, wj = ffd.ffd_plan_describe(planner, ffd.FFD_OP_CROSS, q2, d2, 2)
    assert sm["per_lane"] == 0
    plan_sim.check(sm, jobs, wj, (q2, d2), range(501 * 401))
