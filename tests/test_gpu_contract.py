"""GPU checks of the memory contract of the C ABI (include/ffd.h): every
eager call writes its plan into the workspace, so a workspace whose contents
changed between calls gives the same results; long single pairs and the
search calls run in scratch the caller registers (the library allocates no
device memory); calls on different streams that share the context's memory
are ordered."""
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


def test_workspace_cleared_between_identical_calls(ctx):
    """Two identical ffd_batch calls on one caller workspace, with the
    workspace zero-filled in between (as if torch had handed the block to
    other work): the second call must not rely on what the first left."""
    from paper_2404_05708_amd import ffd
    say("case: workspace zero-filled between two identical batch calls")
    P, p_off, Q, q_off = workloads.random_pairs(61, 300, 1, 2600, dim=2)
    ws = torch.empty(ctx.workspace_size(ffd.FFD_OP_BATCH, p_off, q_off, 2), dtype=torch.uint8, device="cuda:0")
    Pd, Qd = dev(P), dev(Q)
    ctx.set_split(1e-9)  # split every multi-band pair: job table, flags and links all matter
    try:
        first = ctx.batch(Pd, p_off, Qd, q_off, workspace=ws).cpu().numpy()
        assert ctx.last_errors() == 0
        ws.zero_()
        second = ctx.batch(Pd, p_off, Qd, q_off, workspace=ws).cpu().numpy()
        assert ctx.last_errors() == 0
    finally:
        ctx.set_split(0.0)
    np.testing.assert_array_equal(first, second)
    want = oracle.dfd_batch(P, p_off, Q, q_off, nthreads=16)
    assert np.all(np.abs(second - want) <= TOL * want)


def test_cross_workspace_cleared_between_calls(ctx):
    from paper_2404_05708_amd import ffd
    say("case: cross int, workspace zero-filled between calls")
    Qi, qo, Di, do = workloads.cross_int(seed=62, nq=5, ndb=40, length=300)
    ws = torch.empty(ctx.workspace_size(ffd.FFD_OP_CROSS, qo, do, 2), dtype=torch.uint8, device="cuda:0")
    first = ctx.cross_i32(dev(Qi), qo, dev(Di), do, workspace=ws).cpu().numpy()
    ws.zero_()
    second = ctx.cross_i32(dev(Qi), qo, dev(Di), do, workspace=ws).cpu().numpy()
    np.testing.assert_array_equal(first, second)
    np.testing.assert_array_equal(second, oracle.dfd_cross_i32(Qi, qo, Di, do, nthreads=16))


def test_long_pair_needs_registered_scratch(ctx):
    """A pair split over many wavefronts runs in the scratch the caller
    registers: without it the C call returns FFD_E_NOMEM and launches
    nothing; with it the result matches the oracle, also after the scratch
    was zero-filled."""
    import ctypes
    from paper_2404_05708_amd import ffd
    say("case: long pair through the C ABI with and without scratch")
    rng = np.random.default_rng(63)
    p = workloads.walk(rng, 6000, 2)
    q = workloads.walk(rng, 5000, 2)
    h = ffd.ffd_create(0)
    try:
        pd, qd = dev(p), dev(q)
        out = torch.full((1,), -1.0, dtype=torch.float32, device="cuda:0")
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        args = (h, ctypes.c_void_p(pd.data_ptr()), len(p), ctypes.c_void_p(qd.data_ptr()), len(q), 2, 0,
                ctypes.c_void_p(out.data_ptr()), st)
        need = ffd.ffd_workspace_size(h, ffd.FFD_OP_PAIR, [0, len(p)], [0, len(q)], 2)
        assert need > 0
        assert ffd.lib.ffd_distance(*args) == ffd.FFD_E_NOMEM
        torch.cuda.synchronize()
        assert out.item() == -1.0
        scratch = torch.empty(need, dtype=torch.uint8, device="cuda:0")
        ffd.ffd_set_scratch(h, scratch)
        assert ffd.lib.ffd_distance(*args) == ffd.FFD_OK
        first = out.item()
        assert ffd.ffd_last_errors(h) == 0
        scratch.zero_()
        assert ffd.lib.ffd_distance(*args) == ffd.FFD_OK
        assert ffd.ffd_last_errors(h) == 0
        assert out.item() == first
        want = oracle.dfd(p, q, oracle.EUCLIDEAN, "rolling")
        assert abs(first - want) <= TOL * want
        # short pairs need no scratch at all
        assert ffd.ffd_workspace_size(h, ffd.FFD_OP_PAIR, [0, 100], [0, 90], 2) == 0
        torch.cuda.synchronize()
    finally:
        ffd.ffd_destroy(h)


def test_search_needs_registered_scratch(ctx):
    import ctypes
    from paper_2404_05708_amd import ffd
    say("case: decider through the C ABI with and without scratch")
    P, p_off, Q, q_off = workloads.random_pairs(64, 40, 1, 900, dim=2)
    h = ffd.ffd_create(0)
    try:
        Pd, Qd = dev(P), dev(Q)
        out = torch.empty(40, dtype=torch.float32, device="cuda:0")
        po, qo = np.asarray(p_off, dtype=np.int64), np.asarray(q_off, dtype=np.int64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        args = (h, ctypes.c_void_p(Pd.data_ptr()), po.ctypes.data_as(i64p), ctypes.c_void_p(Qd.data_ptr()),
                qo.ctypes.data_as(i64p), 40, 2, 0, ctypes.c_float(np.inf), ctypes.c_void_p(out.data_ptr()), st)
        assert ffd.lib.ffd_decide_batch(*args) == ffd.FFD_E_NOMEM
        need = ffd.ffd_workspace_size(h, ffd.FFD_OP_DECIDE, p_off, q_off, 2)
        scratch = torch.empty(need, dtype=torch.uint8, device="cuda:0")
        ffd.ffd_set_scratch(h, scratch)
        assert ffd.lib.ffd_decide_batch(*args) == ffd.FFD_OK
        got = out.cpu().numpy()
        want = oracle.dfd_batch(P, p_off, Q, q_off, nthreads=16)
        assert np.all(np.abs(got - want) <= TOL * want)
        torch.cuda.synchronize()
    finally:
        ffd.ffd_destroy(h)


def test_shared_workspace_across_streams(ctx):
    """Calls without an explicit workspace share the context's own one; a call
    on a second stream right after one on the first must wait for it (the
    library orders them), so both results are right."""
    say("case: two streams, the context's workspace, different offsets")
    A = workloads.random_pairs(65, 200, 1, 2500, dim=2)
    B = workloads.random_pairs(66, 150, 1, 2500, dim=2)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    dA = (dev(A[0]), A[1], dev(A[2]), A[3])
    dB = (dev(B[0]), B[1], dev(B[2]), B[3])
    torch.cuda.synchronize()
    ctx.set_split(1e-9)
    try:
        outs = []
        for _ in range(3):
            with torch.cuda.stream(s1):
                oa = ctx.batch(*dA, stream=s1)
            with torch.cuda.stream(s2):
                ob = ctx.batch(*dB, stream=s2)
            outs.append((oa, ob))
        torch.cuda.synchronize()
    finally:
        ctx.set_split(0.0)
    wa = oracle.dfd_batch(A[0], A[1], A[2], A[3], nthreads=16)
    wb = oracle.dfd_batch(B[0], B[1], B[2], B[3], nthreads=16)
    for oa, ob in outs:
        a, b = oa.cpu().numpy(), ob.cpu().numpy()
        assert np.all(np.abs(a - wa) <= TOL * wa)
        assert np.all(np.abs(b - wb) <= TOL * wb)
