"""Launches recorded into a HIP graph by stream capture, and repeated linked
launches.

A recorded launch must give, at every replay, the same bits as the same call
made outside the graph, also when its bands hand boundary rows to each other
through progress flags (every replay reuses the recorded epoch, so the flags
are cleared by a recorded kernel first).  Each replay is separated from the
next by the program's own work on the device and a synchronisation.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

REPLAYS = 4


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


def workspace(ctx, ffd, op, a_off, b_off, dim):
    return torch.empty(max(ctx.workspace_size(op, a_off, b_off, dim), 1), dtype=torch.uint8, device="cuda:0")


def replay_and_compare(ctx, g, out, eager, inputs=None):
    """Replay `g` REPLAYS times.  With `inputs` = [(tensor, (a, b)), ...] the
    recorded input buffers alternate between two contents a and b, and
    `eager` = (result for a, result for b): a replay that started from the
    previous replay's progress flags would read boundary rows of the other
    input before they are rewritten."""
    for k in range(REPLAYS):
        want = eager
        if inputs is not None:
            for buf, alt in inputs:
                buf.copy_(alt[k % 2])
            want = eager[k % 2]
        out.fill_(-1)  # the program's own work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert ctx.last_errors() == 0, k
        assert torch.equal(out, want), k


def other(a):
    """The same curves moved and stretched: other distances, same shapes."""
    return (a * np.float32(1.25) + np.float32(3.0)).astype(a.dtype)


def test_batch_replays_equal_eager(ctx, ffdmod):
    P, p_off, Q, q_off = workloads.random_pairs(60, 300, 1, 900, dim=2)
    Pd, Qd = dev(P), dev(Q)
    out = torch.empty(len(p_off) - 1, dtype=torch.float32, device="cuda:0")
    ws = workspace(ctx, ffdmod, ffdmod.FFD_OP_BATCH, p_off, q_off, 2)
    say("case: graph, batch of 300 pairs, eager call")
    ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws)
    torch.cuda.synchronize()
    eager = out.clone()
    assert np.all(np.abs(eager.cpu().numpy() - oracle.dfd_batch(P, p_off, Q, q_off, nthreads=8))
                  <= 2e-6 * oracle.dfd_batch(P, p_off, Q, q_off, nthreads=8))
    g = torch.cuda.CUDAGraph()
    say("case: graph, batch capture")
    with torch.cuda.graph(g):
        ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws)
    say("case: graph, batch replays")
    replay_and_compare(ctx, g, out, eager)


def test_linked_batch_replays_equal_eager(ctx, ffdmod):
    """Every multi-band pair split over waves: boundary rows travel through
    global links whose flags the replays must see cleared."""
    P, p_off, Q, q_off = workloads.random_pairs(61, 40, 300, 2500, dim=2)
    Pd, Qd = dev(P), dev(Q)
    alts = [(Pd, (dev(P), dev(other(P)))), (Qd, (dev(Q), dev(other(Q))))]
    out = torch.empty(len(p_off) - 1, dtype=torch.float32, device="cuda:0")
    ctx.set_tuning(2, 0)
    ctx.set_split(1e-9)
    try:
        ws = workspace(ctx, ffdmod, ffdmod.FFD_OP_BATCH, p_off, q_off, 2)
        say("case: graph, linked batch, eager calls")
        eager = []
        for k in range(2):
            for buf, alt in alts:
                buf.copy_(alt[k])
            ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws)
            torch.cuda.synchronize()
            assert ctx.last_errors() == 0
            eager.append(out.clone())
        assert not torch.equal(eager[0], eager[1])
        g = torch.cuda.CUDAGraph()
        say("case: graph, linked batch capture")
        with torch.cuda.graph(g):
            ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws)
        say("case: graph, linked batch replays")
        replay_and_compare(ctx, g, out, eager, alts)
    finally:
        ctx.set_split(0.0)
        ctx.set_tuning(0, 0)
    for k, (PP, QQ) in enumerate([(P, Q), (other(P), other(Q))]):
        want = oracle.dfd_batch(PP, p_off, QQ, q_off, nthreads=8)
        assert np.all(np.abs(eager[k].cpu().numpy() - want) <= 2e-6 * want)


def test_pipelined_pair_and_int_cross_replays(ctx, ffdmod):
    rng = np.random.default_rng(62)
    p = workloads.walk(rng, 64 * 4 * 6 + 7, 2)
    q = workloads.walk(rng, 1800, 2)
    pd, qd = dev(p), dev(q)
    alts = [(pd, (dev(p), dev(other(p)))), (qd, (dev(q), dev(other(q))))]
    out = torch.empty(1, dtype=torch.float32, device="cuda:0")
    ctx.set_tuning(4, 0)
    try:
        say("case: graph, pipelined pair, eager calls")
        eager = []
        for k in range(2):
            for buf, alt in alts:
                buf.copy_(alt[k])
            ctx.distance(pd, qd, out=out)
            torch.cuda.synchronize()
            assert ctx.last_errors() == 0
            eager.append(out.clone())
        assert eager[0].item() == oracle.dfd_f32_replica(p, q)
        assert eager[1].item() == oracle.dfd_f32_replica(other(p), other(q))
        g = torch.cuda.CUDAGraph()
        say("case: graph, pipelined pair capture")
        with torch.cuda.graph(g):
            ctx.distance(pd, qd, out=out)
        say("case: graph, pipelined pair replays")
        replay_and_compare(ctx, g, out, eager, alts)
    finally:
        ctx.set_tuning(0, 0)
    Qi, qoi, Di, doi = workloads.cross_int(seed=63, nq=5, ndb=40, length=300)
    Qd, Dd = dev(Qi), dev(Di)
    outi = torch.empty(5 * 40, dtype=torch.int64, device="cuda:0")
    ws = workspace(ctx, ffdmod, ffdmod.FFD_OP_CROSS, qoi, doi, 2)
    say("case: graph, int cross, eager call")
    ctx.cross_i32(Qd, qoi, Dd, doi, out=outi, workspace=ws)
    torch.cuda.synchronize()
    eager = outi.clone()
    np.testing.assert_array_equal(eager.cpu().numpy().reshape(5, 40),
                                  oracle.dfd_cross_i32(Qi, qoi, Di, doi, nthreads=8))
    g = torch.cuda.CUDAGraph()
    say("case: graph, int cross capture")
    with torch.cuda.graph(g):
        ctx.cross_i32(Qd, qoi, Dd, doi, out=outi, workspace=ws)
    say("case: graph, int cross replays")
    replay_and_compare(ctx, g, outi, eager)


def test_capture_without_resident_plan_is_refused(ctx, ffdmod):
    P, p_off, Q, q_off = workloads.random_pairs(64, 20, 1, 600, dim=3)
    Pd, Qd = dev(P), dev(Q)
    out = torch.empty(len(p_off) - 1, dtype=torch.float32, device="cuda:0")
    ws = workspace(ctx, ffdmod, ffdmod.FFD_OP_BATCH, p_off, q_off, 3)
    torch.cuda.synchronize()
    say("case: graph, capture of a call whose plan is not resident")
    g = torch.cuda.CUDAGraph()
    with pytest.raises(ffdmod.FFDError) as ei:
        with torch.cuda.graph(g):
            ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws)
    assert ei.value.status == ffdmod.FFD_E_UNSUPPORTED
    torch.cuda.synchronize()
    # the same call outside the capture still works
    got = ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws).cpu().numpy()
    want = oracle.dfd_batch(P, p_off, Q, q_off, nthreads=8)
    assert np.all(np.abs(got - want) <= 2e-6 * want)


def test_repeated_linked_launches_are_bit_identical(ctx):
    """100 launches of a plan whose waves wait on each other's progress
    flags, and 20 of a pipelined pair: every launch gives the same bits."""
    P, p_off, Q, q_off = workloads.random_pairs(65, 50, 500, 2200, dim=2)
    Pd, Qd = dev(P), dev(Q)
    ctx.set_tuning(1, 0)
    ctx.set_split(1e-9)
    try:
        say("case: 100 linked batch launches")
        first = ctx.batch(Pd, p_off, Qd, q_off)
        outs = [ctx.batch(Pd, p_off, Qd, q_off) for _ in range(99)]
        torch.cuda.synchronize()
        assert ctx.last_errors() == 0
        for o in outs:
            assert torch.equal(o, first)
    finally:
        ctx.set_split(0.0)
        ctx.set_tuning(0, 0)
    rng = np.random.default_rng(66)
    p = workloads.walk(rng, 64 * 2 * 9 + 3, 3)
    q = workloads.walk(rng, 2100, 3)
    pd, qd = dev(p), dev(q)
    ctx.set_tuning(2, 0)
    try:
        say("case: 20 pipelined pair launches")
        vals = [ctx.distance(pd, qd) for _ in range(20)]
        torch.cuda.synchronize()
        assert ctx.last_errors() == 0
    finally:
        ctx.set_tuning(0, 0)
    want = oracle.dfd_f32_replica(p, q)
    assert all(v.item() == want for v in vals)
