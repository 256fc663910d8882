"""Stress of the wave-to-wave hand-offs: the debug build of the streaming
kernels (libffd_jitter.so, FFD_DEBUG_JITTER) pauses for a pseudo-random
time before every progress publication -- link counts in global memory and
LDS-ring counters -- so the waits on them resolve in other orders than in
the release build.  Split batches (links between waves) and a long single
pair (the planner's band pipeline) must give the release library's bits,
repeatedly, with no error flags."""
import ctypes
import os

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_jitter_build_matches_release(gpu):
    from paper_2404_05708_amd import ffd
    path = os.path.join(ROOT, "paper_2404_05708_amd", "libffd_jitter.so")
    jl = ffd.load_library(path)
    dev = torch.device("cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ctx = ffd.Context(0)
    h = ctypes.c_void_p()
    assert jl.ffd_create(0, ctypes.byref(h)) == ffd.FFD_OK
    flags = ctypes.c_int32()
    try:
        P, p_off, Q, q_off = workloads.random_pairs(900, 200, 1, 3000, dim=2)
        Pd, Qd = torch.from_numpy(P).to(dev), torch.from_numpy(Q).to(dev)
        base = ctx.batch(Pd, p_off, Qd, q_off).cpu().numpy()
        po = np.ascontiguousarray(p_off, dtype=np.int64)
        qo = np.ascontiguousarray(q_off, dtype=np.int64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        pop, qop = po.ctypes.data_as(i64p), qo.ctypes.data_as(i64p)
        npairs = len(po) - 1
        assert jl.ffd_set_tuning(h, 2, 0) == ffd.FFD_OK
        assert jl.ffd_set_split(h, 1e-9) == ffd.FFD_OK
        nbytes = ctypes.c_size_t()
        assert jl.ffd_workspace_size(h, ffd.FFD_OP_BATCH, pop, npairs, qop, npairs, 2,
                                     ctypes.byref(nbytes)) == ffd.FFD_OK
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        out = torch.empty(npairs, dtype=torch.float32, device=dev)
        for rep in range(5):
            print(f"case: jitter split batch, repeat {rep}", flush=True)
            assert jl.ffd_batch(h, ctypes.c_void_p(Pd.data_ptr()), pop, ctypes.c_void_p(Qd.data_ptr()), qop,
                                npairs, 2, ffd.FFD_EUCLIDEAN, ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(ws.data_ptr()), nbytes.value, stream) == ffd.FFD_OK
            assert jl.ffd_last_errors(h, ctypes.byref(flags)) == ffd.FFD_OK and flags.value == 0
            np.testing.assert_array_equal(out.cpu().numpy(), base)
        assert jl.ffd_set_split(h, 0.0) == ffd.FFD_OK
        assert jl.ffd_set_tuning(h, 0, 0) == ffd.FFD_OK
        rng = np.random.default_rng(901)
        p, q = workloads.walk(rng, 24000, 3), workloads.walk(rng, 20000, 3)
        pd, qd = torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev)
        want = ctx.distance(pd, qd).item()
        one = torch.empty(1, dtype=torch.float32, device=dev)
        # the pipelined pair runs in scratch the caller registers
        pair_off = [np.array([0, 24000], dtype=np.int64), np.array([0, 20000], dtype=np.int64)]
        assert jl.ffd_workspace_size(h, ffd.FFD_OP_PAIR, pair_off[0].ctypes.data_as(i64p), 1,
                                     pair_off[1].ctypes.data_as(i64p), 1, 3, ctypes.byref(nbytes)) == ffd.FFD_OK
        scratch = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        assert jl.ffd_set_scratch(h, ctypes.c_void_p(scratch.data_ptr()), nbytes.value) == ffd.FFD_OK
        for rep in range(3):
            print(f"case: jitter long pair, repeat {rep}", flush=True)
            assert jl.ffd_distance(h, ctypes.c_void_p(pd.data_ptr()), 24000, ctypes.c_void_p(qd.data_ptr()), 20000,
                                   3, ffd.FFD_EUCLIDEAN, ctypes.c_void_p(one.data_ptr()), stream) == ffd.FFD_OK
            assert jl.ffd_last_errors(h, ctypes.byref(flags)) == ffd.FFD_OK and flags.value == 0
            assert one.item() == want
    finally:
        torch.cuda.synchronize()
        jl.ffd_destroy(h)
        ctx.close()


@pytest.mark.parametrize("dim", [6, 12])
def test_jitter_wide_split_batch(gpu, dim):
    """The kernels of 8 and 16 coordinates (curves of 5 to 16) under the
    same pauses: a batch split into bands over waves gives the release
    bits, repeatedly, with no error flags."""
    from paper_2404_05708_amd import ffd
    path = os.path.join(ROOT, "paper_2404_05708_amd", "libffd_jitter.so")
    jl = ffd.load_library(path)
    dev = torch.device("cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ctx = ffd.Context(0)
    h = ctypes.c_void_p()
    assert jl.ffd_create(0, ctypes.byref(h)) == ffd.FFD_OK
    flags = ctypes.c_int32()
    try:
        P, p_off, Q, q_off = workloads.random_pairs(910 + dim, 80, 1, 1500, dim=dim)
        Pd, Qd = torch.from_numpy(P).to(dev), torch.from_numpy(Q).to(dev)
        base = ctx.batch(Pd, p_off, Qd, q_off).cpu().numpy()
        po = np.ascontiguousarray(p_off, dtype=np.int64)
        qo = np.ascontiguousarray(q_off, dtype=np.int64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        pop, qop = po.ctypes.data_as(i64p), qo.ctypes.data_as(i64p)
        npairs = len(po) - 1
        assert jl.ffd_set_split(h, 1e-9) == ffd.FFD_OK
        nbytes = ctypes.c_size_t()
        assert jl.ffd_workspace_size(h, ffd.FFD_OP_BATCH, pop, npairs, qop, npairs, dim,
                                     ctypes.byref(nbytes)) == ffd.FFD_OK
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        out = torch.empty(npairs, dtype=torch.float32, device=dev)
        for rep in range(3):
            print(f"case: jitter wide split batch dim={dim}, repeat {rep}", flush=True)
            assert jl.ffd_batch(h, ctypes.c_void_p(Pd.data_ptr()), pop, ctypes.c_void_p(Qd.data_ptr()), qop,
                                npairs, dim, ffd.FFD_EUCLIDEAN, ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(ws.data_ptr()), nbytes.value, stream) == ffd.FFD_OK
            assert jl.ffd_last_errors(h, ctypes.byref(flags)) == ffd.FFD_OK and flags.value == 0
            np.testing.assert_array_equal(out.cpu().numpy(), base)
    finally:
        torch.cuda.synchronize()
        jl.ffd_destroy(h)
        ctx.close()
