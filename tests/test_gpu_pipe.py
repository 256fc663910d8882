"""The pipelined single-pair kernel on shapes chosen for its index
arithmetic, forced with waves_per_simd = -1 (the planner would run most of
them on the job-table kernels): several passes (more bands than waves),
column counts around the 16-step group and the 4-column batch, partial last
workgroups, both orientations, D = 1 ... 4, squared cells and FP64-exact
values of int32 coordinates.  Float results must equal the oracle's float
replica bit for bit (the recurrence only selects values), int results the
int64 oracle; no device error flags."""
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


def pipelined(ctx, n, m, dim, exact=False):
    from paper_2404_05708_amd import ffd
    sm, _, _ = ffd.ffd_plan_describe(ctx.handle, ffd.FFD_OP_PAIR, [0, n], [0, m], dim, exact=exact,
                                     metric=1 if exact else 0)
    return sm


# (n, m, dim, R): passes, small and ragged column counts, partial workgroups
CASES = [
    (64 * 2 * 1030 + 17, 333, 2, 2),    # 1031 bands: two passes over 1024 waves
    (64 * 4 * 1026, 100, 3, 4),         # 1026 bands at R = 4
    (5000, 2, 2, 2), (5000, 3, 1, 2), (4000, 17, 4, 2), (3000, 63, 2, 4), (3000, 65, 3, 2),
    (64 * 2 * 9 + 1, 700, 2, 2), (64 * 4 * 6 + 3, 1500, 3, 4), (64 * 2 * 7, 2049, 1, 2),
    (300, 20000, 2, 2),                 # either orientation may hold the rows
    (2000, 1000, 4, 4),
]


@pytest.mark.parametrize("n,m,dim,R", CASES)
def test_pipe_shapes_bit_exact(ctx, n, m, dim, R):
    rng = np.random.default_rng(n * 7 + m)
    p = workloads.walk(rng, n, dim)
    q = workloads.walk(rng, m, dim)
    ctx.set_tuning(R, -1)
    try:
        sm = pipelined(ctx, n, m, dim)
        assert sm["pipelined"] == 1 and sm["rows_per_lane"] == R, sm
        say(f"case: pipe n={n} m={m} D={dim} R={R} waves={sm['waves']}")
        pd, qd = dev(p), dev(q)
        got = ctx.distance(pd, qd).item()
        assert ctx.last_errors() == 0
        got_sq = ctx.distance(pd, qd, metric=1).item()
        assert ctx.last_errors() == 0
    finally:
        ctx.set_tuning(0, 0)
    assert got == oracle.dfd_f32_replica(p, q), (n, m, dim, R)
    assert got_sq == oracle.dfd_f32_replica(p, q, oracle.SQEUCLIDEAN), (n, m, dim, R)


@pytest.mark.parametrize("n,m,dim,R", [(64 * 2 * 6 + 5, 900, 2, 2), (64 * 4 * 5, 1300, 3, 4), (2600, 40, 1, 2)])
def test_pipe_exact_int(ctx, n, m, dim, R):
    rng = np.random.default_rng(n + 3 * m)
    p = rng.integers(-(1 << 15), 1 << 15, size=(n, dim), dtype=np.int32)
    q = rng.integers(-(1 << 15), 1 << 15, size=(m, dim), dtype=np.int32)
    ctx.set_tuning(R, -1)
    try:
        sm = pipelined(ctx, n, m, dim, exact=True)
        assert sm["pipelined"] == 1 and sm["rows_per_lane"] == R, sm
        say(f"case: pipe exact n={n} m={m} D={dim} R={R}")
        got = ctx.distance_i32(dev(p), dev(q)).item()
        assert ctx.last_errors() == 0
    finally:
        ctx.set_tuning(0, 0)
    assert got == oracle.dfd_i32(p, q)
