"""ffd_batch_noalloc (the entry point for callers that cannot allocate
device memory) against ffd_batch, through the C ABI: two calls in a row on a
fresh context, the second with a smaller input, each bit-identical to
ffd_batch on a caller workspace (the same plan and kernel), with no device
error flags, and within 2e-6 of the FP64 oracle."""
import ctypes
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


def _run(ffd, h, P, p_off, Q, q_off, noalloc):
    i64p = ctypes.POINTER(ctypes.c_int64)
    po, qo = np.ascontiguousarray(p_off, np.int64), np.ascontiguousarray(q_off, np.int64)
    npairs = len(po) - 1
    Pd = torch.from_numpy(P).to("cuda:0")
    Qd = torch.from_numpy(Q).to("cuda:0")
    out = torch.full((npairs,), -1.0, dtype=torch.float32, device="cuda:0")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = (h, ctypes.c_void_p(Pd.data_ptr()), po.ctypes.data_as(i64p), ctypes.c_void_p(Qd.data_ptr()),
            qo.ctypes.data_as(i64p), npairs, P.shape[1], 0)
    if noalloc:
        rc = ffd.lib.ffd_batch_noalloc(*args, ctypes.c_void_p(out.data_ptr()), st)
    else:
        nbytes = ffd.ffd_workspace_size(h, ffd.FFD_OP_BATCH, po, qo, P.shape[1])
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
        rc = ffd.lib.ffd_batch(*args, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nbytes, st)
    assert rc == ffd.FFD_OK, ffd.lib.ffd_last_error(h)
    res = out.cpu().numpy()
    assert ffd.ffd_last_errors(h) == 0
    return res


def test_noalloc_matches_batch_twice(gpu):
    from paper_2404_05708_amd import ffd
    h = ffd.ffd_create(0)
    try:
        say("case: noalloc call 1: the 4096-pair batched workload")
        big = workloads.batched()
        got1 = _run(ffd, h, *big, noalloc=True)
        ref1 = _run(ffd, h, *big, noalloc=False)
        np.testing.assert_array_equal(got1, ref1)
        want1 = oracle.dfd_batch(*big, nthreads=16)
        assert np.all(np.abs(got1 - want1) <= TOL * want1)
        say("case: noalloc call 2: 150 smaller pairs, every multi-band pair split")
        small = workloads.random_pairs(71, 150, 1, 1500, dim=2)
        assert ffd.lib.ffd_set_split(h, ctypes.c_float(1e-9)) == ffd.FFD_OK
        got2 = _run(ffd, h, *small, noalloc=True)
        ref2 = _run(ffd, h, *small, noalloc=False)
        np.testing.assert_array_equal(got2, ref2)
        want2 = oracle.dfd_batch(*small, nthreads=16)
        assert np.all(np.abs(got2 - want2) <= TOL * want2)
        torch.cuda.synchronize()
    finally:
        ffd.ffd_destroy(h)
