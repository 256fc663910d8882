"""Benchmark: DP cells/s of the batched discrete Frechet distance on one GPU.

Workload (synthetic, seeded; see workloads.batched): 4096 independent pairs,
lengths n, m uniform in [64, 2048], 2-D float32 random walks, q = p resampled
at rate m/n plus N(0, 0.1^2) noise, Euclidean ground distance.  One step is
one ffd_batch call over all 4096 pairs with the inputs already resident in
device memory.  Cells are algorithmic (sum of n*m; padding not counted).

Printed: one JSON line with the metric, the roofline of the dominant kernel
(VALU issue rate: the path has no contraction and moves O(n+m) bytes per
pair), the same pairs through the one-pair entry point (plain), and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DP cells/s (batched vs plain, 1 GPU) at stated tol; p50/p99 latency at fixed QPS"
TOL = 2e-6
# MI355X: 256 CUs x 4 SIMD x 16 lanes per clock x 2.4 GHz = 3.93e13 VALU lane-ops/s
PEAK_VALU = 256 * 4 * 16 * 2.4e9


def imin(dim):
    """Algorithmic VALU lane-ops per cell without packed FP32: D subtractions,
    one multiply and D-1 FMAs for the squared distance, then min3 and max."""
    return 2 * dim + 2


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-pair comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-pairs", type=int, default=4096, help="pairs in the CPU oracle sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 256 MiB device copy (reference for HBM counter scaling)")
    ap.add_argument("--rows-per-lane", type=int, default=0)
    ap.add_argument("--waves-per-simd", type=int, default=0)
    ap.add_argument("--split", type=float, default=0.0,
                    help="band splitting: 0 auto, < 0 only when needed, > 0 above this share of a wave's load")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the work shards by pairs across GPUs, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2404_05708_amd import ffd

    dev = torch.device("cuda:0")
    P, p_off, Q, q_off = workloads.batched()
    npairs = len(p_off) - 1
    cells = int(np.sum(np.diff(p_off) * np.diff(q_off)))
    dim = P.shape[1]
    Pd = torch.from_numpy(P).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    ctx = ffd.Context(0)
    ctx.set_tuning(args.rows_per_lane, args.waves_per_simd)
    ctx.set_split(args.split)
    nbytes = ctx.workspace_size(ffd.FFD_OP_BATCH, p_off, q_off, dim)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = torch.empty(npairs, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.copy_probe:
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # timed region: K steps, synchronised on both sides
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps

    # kernel-only duration with HIP events on the launch stream
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    info = ctx.last_launch()
    launch_errors = ctx.last_errors()

    # parity of the timed output against stored oracle values
    import json as _json
    g = _json.load(open(os.path.join(ROOT, "tests", "golden", "expected.json")))["batched"]
    res = out.cpu().numpy()
    idx = np.array(g["sample_index"])
    want = np.array(g["euclidean"])
    parity_ok = bool(np.all(np.abs(res[idx] - want) <= TOL * want))

    value = cells / (ms_per_step / 1e3)
    ops = cells * imin(dim)
    achieved = ops / (kern_ms / 1e3)
    roofline = {
        "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU / 1e12,
        "unit": "TVALUop/s", "frac": achieved / PEAK_VALU, "traffic": None,
        "kernel": f"ffd::stream_kernel<{info['rows_per_lane']}, {dim}, float>", "kernel_ms": kern_ms,
        "launch": info,
        "ops_per_cell": imin(dim), "cells_per_launch": cells,
    }

    plain = None
    if not args.no_plain:
        torch.cuda.synchronize()
        pp = [(Pd[p_off[k]:p_off[k + 1]], Qd[q_off[k]:q_off[k + 1]]) for k in range(npairs)]
        outs = torch.empty(npairs, dtype=torch.float32, device=dev)
        for k in range(8):
            ctx.distance(pp[k][0], pp[k][1], out=outs[k:k + 1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(npairs):
            ctx.distance(pp[k][0], pp[k][1], out=outs[k:k + 1])
        torch.cuda.synchronize()
        pw = time.perf_counter() - t1
        plain = {"cells_per_s": cells / pw, "ms": pw * 1e3,
                 "bit_identical_to_batched": bool(torch.equal(outs, out))}

    cpu = None
    if not args.no_cpu:
        import oracle
        cores = min(16, len(os.sched_getaffinity(0)))
        rng = np.random.default_rng(77)
        sample = np.sort(rng.choice(npairs, size=args.cpu_pairs, replace=False))
        s_cells = int(np.sum((np.diff(p_off) * np.diff(q_off))[sample]))
        ps, pl = p_off[:-1][sample], np.diff(p_off)[sample]
        qs, ql = q_off[:-1][sample], np.diff(q_off)[sample]
        order = np.argsort(-(pl * ql))
        t2 = time.perf_counter()
        vals = oracle.dfd_pairs(P, ps, pl, Q, qs, ql, oracle.EUCLIDEAN, cores, order)
        cw = time.perf_counter() - t2
        agree = bool(np.all(np.abs(res[sample] - vals) <= TOL * vals))
        cpu = {"value": s_cells / cw, "unit": "cells/s", "cores": cores, "kind": "oracle",
               "sample": f"{args.cpu_pairs} of the 4096 pairs (seed 77), {s_cells} cells, FP64 rolling-row "
                         f"oracle, longest first on {cores} threads, {cw:.2f} s",
               "gpu_matches_sample": agree}

    line = {
        "metric": METRIC, "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched: 4096 pairs, n and m uniform in [64, 2048], 2-D float32 "
                               "random walks, q = p resampled + N(0, 0.1^2), Euclidean (seed 2)",
                   "npairs": npairs, "cells": cells, "global_batch": npairs},
        "parity": {"tolerance": TOL, "sampled_ok": parity_ok, "launch_error_flags": launch_errors},
        "roofline": roofline, "plain": plain, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
