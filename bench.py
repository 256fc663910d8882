"""Benchmark: DP cells/s of the discrete Frechet distance on one GPU.

Default workload (the headline line): 4096 independent pairs, lengths n, m
uniform in [64, 2048], 2-D float32 random walks, q = p resampled at rate m/n
plus N(0, 0.1^2) noise, Euclidean ground distance (workloads.batched).  One
step is one ffd_batch call over all 4096 pairs with the inputs already
resident in device memory.  Cells are algorithmic (sum of n*m; padding is
not counted).

--workload selects the other configurations:
  plain  one 512 x 384 2-D pair through ffd_distance (one launch per step)
  large  one 131072 x 131072 3-D pair through ffd_distance
  cross  1024 x 1024 curves of 256 int32 2-D points through ffd_cross_i32
         (squared Euclidean, int64 results, bit-exact)
  serving  Poisson-arrival queries against a resident 10,000-curve database
         through the ffd_server calls: p50/p99 latency at a fixed rate
  dtw    DTW (Appendix B) with squared Euclidean cells on the batched pairs
  levenshtein  Levenshtein distance (Appendix B) of 4096 int32 symbol pairs
  geo    4096 pairs of (latitude, longitude) walks on the sphere under the
         great-circle distance (metric FFD_HAVERSINE)
  decide the decider (ffd_decide_batch) on the batched pairs at the median
         distance
  knn    k = 10 nearest curves of queries in the serving database
         (ffd_knn: bounds, threshold, early-abandoning sweep) against a
         full scan

The batched and short-pairs lines time HIP graph replays of the call
(inputs and the call's plan resident in device memory, the replays' bits
checked against the eager call's); the eager calls' rate, with the plan
uploaded from host memory on every call, is printed beside it ("eager").

Printed: one JSON line with the metric, the roofline of the dominant kernel
(VALU issue rate: the path has no contraction and moves O(n+m) bytes per
pair), and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
# HIP maps a process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 by
# default, round robin in creation order).  The serving block keeps its
# launch slots' streams busy at once; with 4 queues two of them can land on
# one queue and run one after the other, depending on the streams created
# before (measured: saturation 1,200 requests/s after the batched block's
# graph replays, 1,490 without them, 1,650 with 8 queues in either case; the
# other blocks unchanged).  Raised to 8 where the environment sets fewer,
# before the HIP runtime starts; the line records both.
ENV_HW_QUEUES = os.environ.get("GPU_MAX_HW_QUEUES")
if not (ENV_HW_QUEUES or "").isdigit() or int(ENV_HW_QUEUES) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"
HW_QUEUES = {"gpu_max_hw_queues": os.environ["GPU_MAX_HW_QUEUES"], "environment": ENV_HW_QUEUES}
sys.path.insert(0, ROOT)

METRIC = "DP cells/s (batched vs plain, 1 GPU) at stated tol; p50/p99 latency at fixed QPS"
TOL = 2e-6
# MI355X: 256 CUs x 4 SIMD x 16 lanes per clock x 2.4 GHz = 3.93e13 VALU lane-ops/s
# (FP32 without packed math, and FP64: both 16 lanes per SIMD per clock)
PEAK_VALU = 256 * 4 * 16 * 2.4e9


def imin(dim, exact=False, cell="euclidean"):
    """Algorithmic VALU lane-ops per cell without packed FP32: D subtractions,
    one multiply and D-1 FMAs for the squared distance, then the selection:
    min3 and max in FP32; FP64 has no three-input min, so two mins and a max.
    Manhattan cells: D subtractions and D-1 additions (absolute values are
    free source modifiers); Chebyshev: D subtractions and ceil((D-1)/2)
    three-input maxima.  DTW replaces the max by an add (same count)."""
    sel = 3 if exact else 2
    if cell == "levenshtein":
        # a compare per symbol coordinate, then the least of the three
        # neighbours (three-input min), +1, and the select of the diagonal
        # on a match (neighbouring values differ by at most one)
        return dim + 3
    if cell == "manhattan":
        return 2 * dim - 1 + sel
    if cell == "chebyshev":
        return dim + dim // 2 + sel
    return 2 * dim + sel


def time_steps(step, steps, sync):
    # Python's cyclic garbage collector can pause the host for milliseconds
    # in the middle of the loop (each call builds a few small objects):
    # collect before the timed region and keep it off during it
    gc.collect()
    gc.disable()
    try:
        sync()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        sync()
        return (time.perf_counter() - t0) / steps
    finally:
        gc.enable()


def kernel_ms(torch, step, steps, stream, ctx=None):
    """Average duration of one step's launch.  The library's own event pair
    on the launch stream when it records one per step (its kernels alone,
    without the plan upload); otherwise HIP events recorded on the stream
    around each step."""
    if ctx is not None:
        torch.cuda.synchronize()
        ctx.set_kernel_timing(True)
        try:
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            ms, n = ctx.kernel_time()
        finally:
            ctx.set_kernel_timing(False)
        if n == steps:
            return ms / n
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


def graph_replay(torch, call, steps, out):
    """Time one call recorded into a HIP graph: (seconds per replay, whether
    every replay's results equal the eager call's bits).  The eager call
    just before the capture leaves the call's plan (the job table and the
    offsets, from host memory) in the workspace, so a replay runs the
    kernels on inputs and plan already resident in device memory: no
    transfer from host memory inside the timed region."""
    call(None)  # eager, on the current stream
    torch.cuda.synchronize()
    eager = out.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call(None)  # torch's capture stream is current inside the block
    same = True
    for _ in range(2):
        out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same = same and torch.equal(out, eager)
    sec = time_steps(g.replay, steps, torch.cuda.synchronize)
    same = same and torch.equal(out, eager)
    del g
    return sec, same


def resident(cells, sec, gsec, same):
    """The line's rate: graph replays (inputs and plan resident) when their
    bits equal the eager call's, with the eager call's rate beside it."""
    use = gsec if same else sec
    return use, {"ms_per_step": sec * 1e3, "cells_per_s": cells / sec,
                 "note": "one eager call per step: the plan (job table and offsets from host memory) is uploaded "
                         "on every call, inside the timed region"}, \
        {"timing": "HIP graph replay of one call (plan resident in the workspace)" if same else
                   "eager calls (graph replays differed from the eager bits)", "replay_bit_identical": same}


def launch_signature(info):
    return f"R{info['rows_per_lane']}/W{info['waves']}/S{info['stream_steps']}"


def profiled_traffic(profile, info):
    """HBM bytes per launch recorded in a committed rocprofv3 summary
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy), or None when the
    kernel source differs from the one the counters were taken on or the
    planner chose another launch (rows per lane, waves, longest stream)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0].strip() in (
                "kernel_source_sha256", "plan_header_sha256", "launch_signature", "* traffic_bytes_per_launch"):
            k, v = line.split(":", 1)
            fields[k.strip().lstrip("* ")] = v.split()[0]
    src = {"kernel_source_sha256": "paper_2404_05708_amd/csrc/ffd_stream.h",
           "plan_header_sha256": "paper_2404_05708_amd/csrc/ffd_plan.h"}
    for key, rel in src.items():
        digest = hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()
        if fields.get(key) != digest:
            return None
    if fields.get("launch_signature") != launch_signature(info):
        return None
    return float(fields["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in fields else None


def kernel_dim(dim):
    """Coordinates per point of the kernel that runs curves of `dim`."""
    return dim if dim <= 4 else (8 if dim <= 8 else 16)


def roofline(info, cells, kms, dim, exact, profile=None, family="stream_kernel", suffix="", cell="euclidean"):
    ops = cells * imin(dim, exact, cell)
    achieved = ops / (kms / 1e3)
    vt = "double" if exact else "float"
    return {
        "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU / 1e12,
        "unit": "TVALUop/s", "frac": achieved / PEAK_VALU,
        "traffic": profiled_traffic(profile, info) if profile else None,
        "kernel": f"ffd::{family}<{info['rows_per_lane']}, {kernel_dim(dim)}, {vt}{suffix}>", "kernel_ms": kms,
        "launch": info, "ops_per_cell": imin(dim, exact, cell), "cells_per_launch": cells,
    }


def golden():
    return json.load(open(os.path.join(ROOT, "tests", "golden", "expected.json")))


def cpu_cores():
    """Threads the oracle runs on: every core this process may use, within
    the host's CPU share for one GPU where the environment states it
    (OMP_NUM_THREADS)."""
    n = len(os.sched_getaffinity(0))
    share = os.environ.get("OMP_NUM_THREADS", "")
    return min(n, int(share)) if share.isdigit() and int(share) > 0 else n


def cpu_host():
    """The host the CPU baseline ran on: nproc and the model name."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"), "cpu_model": model}


# ------------------------------------------------------------------ workloads

def run_batched(args, torch, ffd, ctx, dev, stream):
    import workloads
    P, p_off, Q, q_off = workloads.batched(dim=args.dim)
    npairs = len(p_off) - 1
    cells = int(np.sum(np.diff(p_off) * np.diff(q_off)))
    dim = P.shape[1]
    wide = dim != 2  # the same lengths with other dimensions: no stored values, no profile
    Pd = torch.from_numpy(P).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    nbytes = ctx.workspace_size(ffd.FFD_OP_BATCH, p_off, q_off, dim)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = torch.empty(npairs, dtype=torch.float32, device=dev)
    metric = {"euclidean": ffd.FFD_EUCLIDEAN, "manhattan": ffd.FFD_MANHATTAN,
              "chebyshev": ffd.FFD_CHEBYSHEV}[args.metric]

    def call(st):
        ctx.batch(Pd, p_off, Qd, q_off, metric=metric, out=out, workspace=ws, stream=st)

    def step():
        call(stream)

    tuning = None
    if args.autotune:
        tuning = ctx.autotune_batch(Pd, p_off, Qd, q_off, metric=metric, out=out, workspace=ws, stream=stream)
    for _ in range(args.warmup):
        step()
    if args.copy_probe:
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sec = time_steps(step, args.steps, torch.cuda.synchronize)
    kms = kernel_ms(torch, step, args.steps, stream, ctx)
    info = ctx.last_launch()
    errs = ctx.last_errors()
    res = out.cpu().numpy()
    gsec, gsame = graph_replay(torch, call, args.steps, out)
    use, eager, timing = resident(cells, sec, gsec, gsame)
    if wide:
        # 64 pairs of the batch against the FP64 oracle, computed here
        import oracle
        idx = np.sort(np.random.default_rng(78).choice(npairs, size=64, replace=False))
        want = oracle.dfd_pairs(P, p_off[:-1][idx], np.diff(p_off)[idx], Q, q_off[:-1][idx], np.diff(q_off)[idx],
                                metric, cpu_cores())
    else:
        g = golden()["batched" if args.metric == "euclidean" else "batched_" + args.metric]
        idx = np.array(g["sample_index"])
        want = np.array(g[args.metric])
    parity_ok = bool(np.all(np.abs(res[idx] - want) <= TOL * want))

    plain = None
    if not args.no_plain and args.metric == "euclidean" and not wide:
        pp = [(Pd[p_off[k]:p_off[k + 1]], Qd[q_off[k]:q_off[k + 1]]) for k in range(npairs)]
        outs = torch.empty(npairs, dtype=torch.float32, device=dev)
        for k in range(8):
            ctx.distance(pp[k][0], pp[k][1], out=outs[k:k + 1], stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(npairs):
            ctx.distance(pp[k][0], pp[k][1], out=outs[k:k + 1], stream=stream)
        torch.cuda.synchronize()
        pw = time.perf_counter() - t1
        plain = {"cells_per_s": cells / pw, "ms": pw * 1e3,
                 "bit_identical_to_batched": bool(torch.equal(outs, out))}

    cpu = None
    if not args.no_cpu:
        import oracle
        cores = cpu_cores()
        rng = np.random.default_rng(77)
        sample = np.sort(rng.choice(npairs, size=args.cpu_pairs, replace=False))
        s_cells = int(np.sum((np.diff(p_off) * np.diff(q_off))[sample]))
        ps, pl = p_off[:-1][sample], np.diff(p_off)[sample]
        qs, ql = q_off[:-1][sample], np.diff(q_off)[sample]
        order = np.argsort(-(pl * ql))
        t2 = time.perf_counter()
        vals = oracle.dfd_pairs(P, ps, pl, Q, qs, ql, metric, cores, order)
        cw = time.perf_counter() - t2
        agree = bool(np.all(np.abs(res[sample] - vals) <= TOL * vals))
        cpu = {"value": s_cells / cw, "unit": "cells/s", "cores": cores, "kind": "oracle",
               "sample": f"{args.cpu_pairs} of the 4096 pairs (seed 77), {s_cells} cells, FP64 rolling-row "
                         f"oracle, longest first on {cores} threads, {cw:.2f} s",
               "gpu_matches_sample": agree}
    return {
        "value": cells / use, "ms_per_step": use * 1e3, "dtype": "f32", "timing": timing, "eager": eager,
        "config": {"workload": f"batched: 4096 pairs, n and m uniform in [64, 2048], {dim}-D float32 "
                               f"random walks, q = p resampled + N(0, 0.1^2), {args.metric.capitalize()} (seed 2)",
                   "npairs": npairs, "cells": cells, "global_batch": npairs},
        "parity": {"tolerance": TOL, "sampled_ok": parity_ok, "launch_error_flags": errs},
        "autotune": tuning,
        "roofline": (roofline(info, cells, kms, dim, False, None if wide else "stream_kernel_batched_4096pairs.md")
                     if args.metric == "euclidean" else
                     roofline(info, cells, kms, dim, False, family="op_kernel",
                              suffix=", 4" if args.metric == "manhattan" else ", 6", cell=args.metric)),
        "plain": plain, "cpu_baseline": cpu,
    }


def run_short(args, torch, ffd, ctx, dev, stream):
    """Many short pairs: the one-pair-per-lane kernel, with the streaming
    kernel's job-table plan timed on the same pairs beside it."""
    import workloads
    lev = args.levenshtein  # the Levenshtein distance of short symbol sequences instead
    if lev:
        P, p_off, Q, q_off = workloads.short_symbol_pairs()
    else:
        P, p_off, Q, q_off = workloads.short_pairs(long_pairs=800 if args.mixed else 0)
    npairs = len(p_off) - 1
    cells = int(np.sum(np.diff(p_off) * np.diff(q_off)))
    dim = P.shape[1]
    Pd = torch.from_numpy(P).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    nbytes = ctx.workspace_size(ffd.FFD_OP_BATCH, p_off, q_off, dim)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = torch.empty(npairs, dtype=torch.int64 if lev else torch.float32, device=dev)
    dtw = args.dtw  # DTW of squared Euclidean cells instead of the Frechet distance

    def call(st):
        if lev:
            ctx.levenshtein_batch(Pd, p_off, Qd, q_off, out=out, workspace=ws, stream=st)
        elif dtw:
            ctx.dtw_batch(Pd, p_off, Qd, q_off, metric=ffd.FFD_SQEUCLIDEAN, out=out, workspace=ws, stream=st)
        else:
            ctx.batch(Pd, p_off, Qd, q_off, out=out, workspace=ws, stream=st)

    def step():
        call(stream)

    for _ in range(args.warmup):
        step()
    sec = time_steps(step, args.steps, torch.cuda.synchronize)
    kms = kernel_ms(torch, step, args.steps, stream, ctx)
    info = ctx.last_launch()
    res = out.cpu().numpy()
    gsec, gsame = graph_replay(torch, call, args.steps, out)
    use, eager, timing = resident(cells, sec, gsec, gsame)
    import oracle
    idx = np.sort(np.random.default_rng(79).choice(npairs, size=256, replace=False))
    if lev:
        want = oracle.lev_pairs(P, p_off[:-1][idx], np.diff(p_off)[idx], Q, q_off[:-1][idx], np.diff(q_off)[idx],
                                cpu_cores())
    elif dtw:
        want = np.array([oracle.dtw(P[p_off[k]:p_off[k + 1]], Q[q_off[k]:q_off[k + 1]], oracle.SQEUCLIDEAN)
                         for k in idx])
    else:
        want = oracle.dfd_pairs(P, p_off[:-1][idx], np.diff(p_off)[idx], Q, q_off[:-1][idx], np.diff(q_off)[idx],
                                oracle.EUCLIDEAN, cpu_cores())
    if lev:  # exact
        parity_ok = bool(np.array_equal(res[idx], want))
    elif dtw:  # float32 sums: within (n + m + 2 D + 2) roundings
        tol = (np.diff(p_off)[idx] + np.diff(q_off)[idx] + 2 * dim + 2) * 2.0 ** -24 * 1.01
        parity_ok = bool(np.all(np.abs(res[idx] - want) <= tol * want))
    else:
        parity_ok = bool(np.all(np.abs(res[idx] - want) <= TOL * want))
    # the streaming kernel on the same pairs: any forced setting keeps the job-table plan
    ctx.set_tuning(0, 2)
    try:
        for _ in range(2):
            step()
        ssec = time_steps(step, args.steps, torch.cuda.synchronize)
        skms = kernel_ms(torch, step, args.steps, stream, ctx)
        sinfo = ctx.last_launch()
        same = bool(np.array_equal(out.cpu().numpy(), res))
        sgsec, sgsame = graph_replay(torch, call, args.steps, out)
        same = same and bool(np.array_equal(out.cpu().numpy(), res))
        suse = sgsec if sgsame else ssec
    finally:
        ctx.set_tuning(args.rows_per_lane, args.waves_per_simd)
    cpu = None
    if not args.no_cpu and not dtw and not lev:
        cores = cpu_cores()
        rng = np.random.default_rng(80)
        sample = np.sort(rng.choice(npairs, size=min(npairs, 65536), replace=False))
        s_cells = int(np.sum((np.diff(p_off) * np.diff(q_off))[sample]))
        t2 = time.perf_counter()
        vals = oracle.dfd_pairs(P, p_off[:-1][sample], np.diff(p_off)[sample], Q, q_off[:-1][sample],
                                np.diff(q_off)[sample], oracle.EUCLIDEAN, cores)
        cw = time.perf_counter() - t2
        cpu = {"value": s_cells / cw, "unit": "cells/s", "cores": cores, "kind": "oracle",
               "sample": f"{len(sample)} of the {npairs} pairs (seed 80), {s_cells} cells, FP64 rolling-row oracle "
                         f"on {cores} threads, {cw:.2f} s",
               "gpu_matches_sample": bool(np.all(np.abs(res[sample] - vals) <= TOL * vals))}
    rl = roofline(info, cells, kms, dim, False, family="lane_kernel", cell="levenshtein" if lev else "euclidean")
    rl["kernel"] = (f"ffd::lane_kernel<1, float, 4, false>" if lev else
                    f"ffd::lane_kernel<2, float, 0, {'true' if dtw else 'false'}>") + " (one launch, column classes 8 .. 64)" + (
        ", then the streaming kernel for the long pairs (kernel_ms covers both)" if args.mixed else "")
    return {
        "metric": "levenshtein_cells_per_second" if lev else METRIC,
        "value": cells / use, "ms_per_step": use * 1e3, "dtype": "f32", "timing": timing, "eager": eager,
        "config": {"workload": (f"short symbol sequences: {npairs} pairs, n and m uniform in [8, 64], int32 symbols "
                                "uniform in [0, 4), Levenshtein (seed 12)") if lev else
                               (("short and long pairs: 262144 pairs with n and m uniform in [8, 64] and 800 with "
                                 "n and m uniform in [300, 1500], shuffled" if args.mixed else
                                 f"short pairs: {npairs} pairs, n and m uniform in [8, 64]")
                                + ", 2-D float32 random walks, "
                                + ("DTW of squared Euclidean cells" if dtw else "Euclidean") + " (seed 11)"),
                   "npairs": npairs, "cells": cells, "global_batch": npairs},
        "parity": {"tolerance": TOL, "sampled_ok": parity_ok, "launch_error_flags": ctx.last_errors(),
                   "streaming_kernel_bit_identical": same},
        "roofline": rl,
        "streaming_kernel": {"cells_per_s": cells / suse, "ms_per_step": suse * 1e3, "kernel_ms": skms,
                             "eager_ms_per_step": ssec * 1e3,
                             "frac": cells * imin(dim, cell="levenshtein" if lev else "euclidean") / (skms / 1e3) / PEAK_VALU,
                             "launch": sinfo},
        "cpu_baseline": cpu,
    }


def run_dtw(args, torch, ffd, ctx, dev, stream):
    """DTW (Appendix B) with squared Euclidean cells on the batched workload."""
    import workloads
    P, p_off, Q, q_off = workloads.batched()
    npairs = len(p_off) - 1
    cells = int(np.sum(np.diff(p_off) * np.diff(q_off)))
    dim = P.shape[1]
    Pd = torch.from_numpy(P).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    nbytes = ctx.workspace_size(ffd.FFD_OP_BATCH, p_off, q_off, dim)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = torch.empty(npairs, dtype=torch.float32, device=dev)
    metric = ffd.FFD_SQEUCLIDEAN

    def step():
        ctx.dtw_batch(Pd, p_off, Qd, q_off, metric=metric, out=out, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    sec = time_steps(step, args.steps, torch.cuda.synchronize)
    kms = kernel_ms(torch, step, args.steps, stream, ctx)
    info = ctx.last_launch()
    errs = ctx.last_errors()
    g = golden()["dtw_batched"]
    res = out.cpu().numpy()
    idx = np.array(g["sample_index"])
    want = np.array(g["sqeuclidean"])
    n_s, m_s = np.diff(p_off)[idx], np.diff(q_off)[idx]
    bound = (n_s + m_s + dim + 2) * 2.0 ** -24 * 1.01
    parity_ok = bool(np.all(np.abs(res[idx] - want) <= bound * want))

    cpu = None
    if not args.no_cpu:
        import oracle
        cores = cpu_cores()
        rng = np.random.default_rng(77)
        sample = np.sort(rng.choice(npairs, size=args.cpu_pairs, replace=False))
        s_cells = int(np.sum((np.diff(p_off) * np.diff(q_off))[sample]))
        ps, pl = p_off[:-1][sample], np.diff(p_off)[sample]
        qs, ql = q_off[:-1][sample], np.diff(q_off)[sample]
        order = np.argsort(-(pl * ql))
        t2 = time.perf_counter()
        vals = oracle.dfd_pairs(P, ps, pl, Q, qs, ql, oracle.SQEUCLIDEAN, cores, order, measure="dtw")
        cw = time.perf_counter() - t2
        b2 = (pl + ql + dim + 2) * 2.0 ** -24 * 1.01
        cpu = {"value": s_cells / cw, "unit": "cells/s", "cores": cores, "kind": "oracle",
               "sample": f"{args.cpu_pairs} of the 4096 pairs (seed 77), {s_cells} cells, FP64 rolling-row "
                         f"DTW oracle, longest first on {cores} threads, {cw:.2f} s",
               "gpu_matches_sample": bool(np.all(np.abs(res[sample] - vals) <= b2 * vals))}
    return {
        "metric": "dtw_cells_per_second", "value": cells / sec, "ms_per_step": sec * 1e3, "dtype": "f32",
        "config": {"workload": "dtw: DTW (Appendix B) with squared Euclidean cells on the batched pairs: "
                               "4096 pairs, n and m uniform in [64, 2048], 2-D float32 random walks (seed 2)",
                   "npairs": npairs, "cells": cells, "global_batch": npairs},
        "parity": {"tolerance": "(n + m + D + 2) 2^-24 relative", "sampled_ok": parity_ok,
                   "launch_error_flags": errs},
        "roofline": roofline(info, cells, kms, dim, False, family="op_kernel", suffix=", 1"),
        "cpu_baseline": cpu,
    }


def run_levenshtein(args, torch, ffd, ctx, dev, stream):
    """Levenshtein distance (Appendix B) on 4096 pairs of 4-letter int32
    symbol sequences with the batched lengths."""
    import workloads
    P, p_off, Q, q_off = workloads.symbol_pairs()
    npairs = len(p_off) - 1
    cells = int(np.sum(np.diff(p_off) * np.diff(q_off)))
    Pd = torch.from_numpy(P).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    ws = torch.empty(ctx.workspace_size(ffd.FFD_OP_BATCH, p_off, q_off, 1), dtype=torch.uint8, device=dev)
    out = torch.empty(npairs, dtype=torch.int64, device=dev)

    def step():
        ctx.levenshtein_batch(Pd, p_off, Qd, q_off, out=out, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    sec = time_steps(step, args.steps, torch.cuda.synchronize)
    kms = kernel_ms(torch, step, args.steps, stream, ctx)
    info = ctx.last_launch()
    errs = ctx.last_errors()
    g = golden()["levenshtein"]
    res = out.cpu().numpy()
    parity_ok = bool(np.array_equal(res[np.array(g["sample_index"])], np.array(g["levenshtein"], dtype=np.int64)))
    cpu = None
    if not args.no_cpu:
        import oracle
        cores = cpu_cores()
        rng = np.random.default_rng(77)
        sample = np.sort(rng.choice(npairs, size=args.cpu_pairs, replace=False))
        s_cells = int(np.sum((np.diff(p_off) * np.diff(q_off))[sample]))
        ps, pl = p_off[:-1][sample], np.diff(p_off)[sample]
        qs, ql = q_off[:-1][sample], np.diff(q_off)[sample]
        order = np.argsort(-(pl * ql))
        t2 = time.perf_counter()
        vals = oracle.lev_pairs(P, ps, pl, Q, qs, ql, cores, order)
        cw = time.perf_counter() - t2
        cpu = {"value": s_cells / cw, "unit": "cells/s", "cores": cores, "kind": "oracle",
               "sample": f"{args.cpu_pairs} of the 4096 pairs (seed 77), {s_cells} cells, int64 rolling-row "
                         f"Levenshtein oracle, longest first on {cores} threads, {cw:.2f} s",
               "gpu_matches_sample": bool(np.array_equal(vals, res[sample]))}
    return {
        "metric": "levenshtein_cells_per_second", "value": cells / sec, "ms_per_step": sec * 1e3, "dtype": "f32",
        "config": {"workload": "levenshtein: 4096 pairs of int32 symbol sequences over 4 letters, lengths "
                               "uniform in [64, 2048], q = p resampled with 10% redrawn (seed 8)",
                   "npairs": npairs, "cells": cells, "global_batch": npairs},
        "parity": {"exact": True, "sampled_ok": parity_ok, "launch_error_flags": errs},
        "roofline": roofline(info, cells, kms, 1, False, family="op_kernel", suffix=", 8", cell="levenshtein"),
        "cpu_baseline": cpu,
    }


def run_geo(args, torch, ffd, ctx, dev, stream, dtw=False):
    """The Frechet distance (or DTW) under the great-circle ground distance
    on 4096 pairs of (latitude, longitude) walks on the sphere with the
    batched lengths; the kernel runs on FP64 unit vectors (D = 3)."""
    import workloads
    P, p_off, Q, q_off = workloads.geo_pairs()
    npairs = len(p_off) - 1
    cells = int(np.sum(np.diff(p_off) * np.diff(q_off)))
    Pd = torch.from_numpy(P).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    ws = torch.empty(ctx.workspace_size(ffd.FFD_OP_BATCH, p_off, q_off, 2), dtype=torch.uint8, device=dev)
    out = torch.empty(npairs, dtype=torch.float32, device=dev)

    fn = ctx.dtw_batch if dtw else ctx.batch

    def step():
        fn(Pd, p_off, Qd, q_off, metric=ffd.FFD_HAVERSINE, out=out, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    sec = time_steps(step, args.steps, torch.cuda.synchronize)
    kms = kernel_ms(torch, step, args.steps, stream, ctx)
    info = ctx.last_launch()
    errs = ctx.last_errors()
    g = golden()["dtw_haversine" if dtw else "batched_haversine"]
    res = out.cpu().numpy()
    want = np.array(g["haversine"])
    absb = 1e-12 * (np.diff(p_off) + np.diff(q_off)) if dtw else 1e-12
    idx = np.array(g["sample_index"])
    parity_ok = bool(np.all(np.abs(res[idx] - want) <= TOL * want + (absb[idx] if dtw else absb)))
    cpu = None
    if not args.no_cpu:
        import oracle
        cores = cpu_cores()
        nsample = min(args.cpu_pairs, 1024)
        rng = np.random.default_rng(77)
        sample = np.sort(rng.choice(npairs, size=nsample, replace=False))
        s_cells = int(np.sum((np.diff(p_off) * np.diff(q_off))[sample]))
        ps, pl = p_off[:-1][sample], np.diff(p_off)[sample]
        qs, ql = q_off[:-1][sample], np.diff(q_off)[sample]
        order = np.argsort(-(pl * ql))
        t2 = time.perf_counter()
        vals = oracle.dfd_pairs(P, ps, pl, Q, qs, ql, oracle.HAVERSINE, cores, order,
                                measure="dtw" if dtw else "dfd")
        cw = time.perf_counter() - t2
        sb = 1e-12 * (pl + ql) if dtw else 1e-12
        cpu = {"value": s_cells / cw, "unit": "cells/s", "cores": cores, "kind": "oracle",
               "sample": f"{nsample} of the 4096 pairs (seed 77), {s_cells} cells, FP64 haversine rolling-row "
                         f"{'DTW ' if dtw else ''}oracle, longest first on {cores} threads, {cw:.2f} s",
               "gpu_matches_sample": bool(np.all(np.abs(res[sample] - vals) <= TOL * vals + sb))}
    return {
        "metric": "geo_dtw_cells_per_second" if dtw else "geo_cells_per_second", "value": cells / sec,
        "ms_per_step": sec * 1e3, "dtype": "f64",
        "config": {"workload": "geo: 4096 pairs of (latitude, longitude) random walks on the sphere, steps "
                               "N(0, (2e-3 rad)^2), n and m uniform in [64, 2048], q = p resampled + "
                               "N(0, (2e-4 rad)^2), great-circle distance" + (", DTW" if dtw else "") +
                               " (seed 9)",
                   "npairs": npairs, "cells": cells, "global_batch": npairs},
        "parity": {"tolerance": "2e-6 relative + 1e-12 rad" + (" per cell of a coupling" if dtw else ""),
                   "sampled_ok": parity_ok, "launch_error_flags": errs},
        "roofline": roofline(info, cells, kms, 3, True, family="op_kernel", suffix=", 11" if dtw else ", 10"),
        "cpu_baseline": cpu,
    }


def run_decide(args, torch, ffd, ctx, dev, stream):
    """The decider on the batched pairs at eps = the median distance of the
    stored sample (about half the pairs answer no): effective cells/s over
    all cells of the workload.  The early-abandoning sweep's own roofline
    comes from the same call at the largest finite float threshold, where
    the sweep runs but drops nothing; at eps = +inf the decider runs the
    streaming batch kernel instead (nothing can be dropped), reported
    beside it."""
    import workloads
    P, p_off, Q, q_off = workloads.batched()
    npairs = len(p_off) - 1
    cells = int(np.sum(np.diff(p_off) * np.diff(q_off)))
    Pd = torch.from_numpy(P).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    out = torch.empty(npairs, dtype=torch.float32, device=dev)
    g = golden()["batched"]
    eps = float(np.median(g["euclidean"]))
    big = float(np.finfo(np.float32).max)

    def step(e):
        return lambda: ctx.decide_batch(Pd, p_off, Qd, q_off, e, out=out, stream=stream)

    for _ in range(args.warmup):
        step(eps)()
    sec = time_steps(step(eps), args.steps, torch.cuda.synchronize)
    kms = kernel_ms(torch, step(eps), args.steps, stream, ctx)
    res = out.cpu().numpy()
    idx = np.array(g["sample_index"])
    want = np.array(g["euclidean"])
    dec_ok = bool(np.all((res[idx] <= eps) == (want <= eps)))
    kept = res[idx] <= eps
    val_ok = bool(np.all(np.abs(res[idx][kept] - want[kept]) <= TOL * want[kept]))
    frac_no = float(np.mean(np.isinf(res)))
    step(big)()
    kms_all = kernel_ms(torch, step(big), args.steps, stream, ctx)
    swept = out.cpu().numpy()
    step(np.inf)()
    sec_inf = time_steps(step(np.inf), args.steps, torch.cuda.synchronize)
    kms_inf = kernel_ms(torch, step(np.inf), args.steps, stream, ctx)
    full = out.cpu().numpy()
    info = {"rows_per_lane": 8, "waves": "1 to 2 per SIMD, one pair per wave at a time"}
    inf_line = roofline(ctx.last_launch(), cells, kms_inf, 2, False)
    return {
        "metric": "decider_effective_cells_per_second", "value": cells / sec, "ms_per_step": sec * 1e3,
        "dtype": "f32",
        "config": {"workload": "decide: the batched pairs (seed 2), is delta <= eps? with eps the median "
                               f"of the stored sample ({eps:.6g})", "npairs": npairs, "cells": cells,
                   "global_batch": npairs},
        "parity": {"decisions_ok": dec_ok, "kept_values_ok": val_ok, "share_answered_no": frac_no,
                   "no_drop_sweep_equals_batch_sample": bool(np.all(np.abs(swept[idx] - want) <= TOL * want)),
                   "no_threshold_equals_batch_sample": bool(np.all(np.abs(full[idx] - want) <= TOL * want))},
        "search": {"kernel_ms": kms, "no_drop_sweep_ms": kms_all, "no_threshold_ms": sec_inf * 1e3,
                   "no_threshold_kernel": inf_line["kernel"], "no_threshold_frac": inf_line["frac"]},
        "roofline": roofline(info, cells, kms_all, 2, False, family="bounded_kernel"),
    }


def run_knn(args, torch, ffd, ctx, dev, stream):
    """k = 10 nearest curves of queries in the resident 10,000-curve database
    (the serving workload) through ffd_knn_batch (endpoint bounds, a
    threshold from 128 exact distances per query, early-abandoning sweep;
    --knn-batch queries per call), against ffd_knn one query at a time and a
    full scan (ffd_cross of the query with every curve, then the 10
    smallest)."""
    import workloads
    K = 10
    B = max(1, args.knn_batch)
    DB, dbo = workloads.serving_db()
    db_points = int(dbo[-1])
    DBd = torch.from_numpy(DB).to(dev)
    nq = (args.warmup + args.steps) * B
    qs = workloads.serving_queries(count=nq)
    batches = []
    for b in range(args.warmup + args.steps):
        Qs, q_off = workloads.concat(qs[b * B:(b + 1) * B])
        batches.append((torch.from_numpy(Qs).to(dev), q_off))
    for b in range(args.warmup):
        ctx.knn_batch(batches[b][0], batches[b][1], DBd, dbo, K, stream=stream)
    torch.cuda.synchronize()
    timed = range(args.warmup, args.warmup + args.steps)
    t0 = time.perf_counter()
    res = [ctx.knn_batch(batches[b][0], batches[b][1], DBd, dbo, K, stream=stream) for b in timed]
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / (args.steps * B)
    counts = ctx.last_search()
    # the same queries one call each (a sample of 20), and a full scan of them
    sample = list(range(args.warmup * B, args.warmup * B + min(20, args.steps * B)))
    qd = {i: torch.from_numpy(qs[i]).to(dev) for i in sample}
    ws = torch.empty(max(ctx.workspace_size(ffd.FFD_OP_CROSS, [0, len(qs[i])], dbo, 2) for i in sample),
                     dtype=torch.uint8, device=dev)
    full = torch.empty(len(dbo) - 1, dtype=torch.float32, device=dev)
    ctx.knn(qd[sample[0]], DBd, dbo, K, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    single = [ctx.knn(qd[i], DBd, dbo, K, stream=stream) for i in sample]
    torch.cuda.synchronize()
    single_sec = (time.perf_counter() - t1) / len(sample)
    t2 = time.perf_counter()
    scans = []
    for i in sample:
        ctx.cross(qd[i], [0, len(qs[i])], DBd, dbo, out=full, workspace=ws, stream=stream)
        d = full.cpu()
        scans.append(torch.topk(d, K, largest=False, sorted=True))
    torch.cuda.synchronize()
    scan_sec = (time.perf_counter() - t2) / len(sample)
    flat_i = torch.cat([r[0].cpu() for r in res]).reshape(-1, K)
    flat_d = torch.cat([r[1].cpu() for r in res]).reshape(-1, K)
    base = args.warmup * B
    same = all(torch.equal(flat_d[i - base], s.values) for i, s in zip(sample, scans))
    same_single = all(torch.equal(flat_i[i - base], r[0].cpu()) and torch.equal(flat_d[i - base], r[1].cpu())
                      for i, r in zip(sample, single))
    cells = sum(len(qs[i]) for i in range(base, base + args.steps * B)) * db_points
    cpu = None
    if not args.no_cpu:
        import oracle
        cores = cpu_cores()
        i = sample[0]
        t3 = time.perf_counter()
        vals = oracle.dfd_cross(qs[i], [0, len(qs[i])], DB, dbo, oracle.EUCLIDEAN, cores)[0]
        cw = time.perf_counter() - t3
        o_i, o_d = oracle.knn(vals, K)
        cpu = {"value": 1.0 / cw, "unit": "queries/s", "cores": cores, "kind": "oracle",
               "sample": f"one query ({len(qs[i])} points) against all 10,000 curves, FP64 rolling-row oracle "
                         f"on {cores} threads, then the 10 smallest: {cw:.2f} s",
               "gpu_matches_sample": bool(np.array_equal(flat_i[i - base].numpy(), o_i))}
    return {
        "metric": "knn_queries_per_second", "value": 1.0 / sec, "unit": "queries/s", "ms_per_step": sec * B * 1e3,
        "dtype": "f32",
        "config": {"workload": "knn: k = 10 nearest of log-normal-length 2-D walk queries in the 10,000-curve "
                               "serving database (seeds 5, 6), Euclidean",
                   "queries": args.steps * B, "queries_per_call": B, "k": K, "db_points": db_points,
                   "global_batch": B},
        "parity": {"distances_equal_full_scan": same, "batch_equals_single_query_calls": same_single},
        "search": {"single_query_ms": single_sec * 1e3, "full_scan_ms": scan_sec * 1e3,
                   "speedup_over_full_scan": scan_sec / sec, "effective_cells_per_s": cells / (sec * args.steps * B),
                   "last_call_counts": counts},
        "cpu_baseline": cpu,
    }


def run_pair(args, torch, ffd, ctx, dev, stream, which):
    import workloads
    if which == "plain":
        p, q = workloads.plain_pair()
        want = golden()["plain_pair"]["euclidean"]
        desc = "plain: one pair, n=512, m=384, 2-D float32 random walks, Euclidean (seed 1)"
    else:
        p, q = workloads.large_pair()
        want = golden()["large_pair"]["euclidean"]
        desc = "large: one pair, n=m=131072, 3-D float32 random walks, Euclidean (seed 3)"
    n, m, dim = p.shape[0], q.shape[0], p.shape[1]
    cells = n * m
    pd = torch.from_numpy(p).to(dev)
    qd = torch.from_numpy(q).to(dev)
    out = torch.empty(1, dtype=torch.float32, device=dev)

    def step():
        ctx.distance(pd, qd, out=out, stream=stream)

    for _ in range(args.warmup):
        step()
    sec = time_steps(step, args.steps, torch.cuda.synchronize)
    kms = kernel_ms(torch, step, args.steps, stream, ctx)
    info = ctx.last_launch()
    errs = ctx.last_errors()
    got = out.item()
    parity_ok = abs(got - want) <= TOL * want

    cpu = None
    if not args.no_cpu:
        import oracle
        if which == "plain":
            reps = 50
            t0 = time.perf_counter()
            for _ in range(reps):
                v = oracle.dfd(p, q, oracle.EUCLIDEAN, "rolling")
            cw = (time.perf_counter() - t0) / reps
            cpu = {"value": cells / cw, "unit": "cells/s", "cores": 1, "kind": "oracle",
                   "sample": f"the whole pair, FP64 rolling-row oracle, mean of {reps} runs, one thread",
                   "latency_ms": cw * 1e3, "gpu_matches": bool(abs(got - v) <= TOL * v)}
        else:
            k = args.cpu_block
            t0 = time.perf_counter()
            oracle.dfd(p[:k], q[:k], oracle.EUCLIDEAN, "rolling")
            cw = time.perf_counter() - t0
            cpu = {"value": k * k / cw, "unit": "cells/s", "cores": 1, "kind": "oracle",
                   "sample": f"leading {k} x {k} points of both curves ({k * k} cells), FP64 rolling-row "
                             f"oracle, one thread (one pair has no parallelism across pairs), {cw:.2f} s"}
    return {
        "value": cells / sec, "ms_per_step": sec * 1e3, "dtype": "f32",
        "config": {"workload": desc, "npairs": 1, "cells": cells, "global_batch": 1},
        "parity": {"tolerance": TOL, "ok": bool(parity_ok), "got": got, "oracle": want,
                   "launch_error_flags": errs},
        "roofline": roofline(info, cells, kms, dim, False,
                             family="pipe_kernel" if info.get("pipelined") else "stream_kernel"),
        "cpu_baseline": cpu,
    }


def run_cross(args, torch, ffd, ctx, dev, stream):
    import workloads
    Qs, qo, DB, dbo = workloads.cross_int()
    nq, ndb, dim = len(qo) - 1, len(dbo) - 1, Qs.shape[1]
    cells = int(np.sum(np.diff(qo))) * int(np.sum(np.diff(dbo)))
    Qd = torch.from_numpy(Qs).to(dev)
    Dd = torch.from_numpy(DB).to(dev)
    nbytes = ctx.workspace_size(ffd.FFD_OP_CROSS, qo, dbo, dim)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = torch.empty(nq * ndb, dtype=torch.int64, device=dev)

    def step():
        ctx.cross_i32(Qd, qo, Dd, dbo, out=out, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    sec = time_steps(step, args.steps, torch.cuda.synchronize)
    kms = kernel_ms(torch, step, args.steps, stream, ctx)
    info = ctx.last_launch()
    errs = ctx.last_errors()
    g = golden()["cross_int"]
    res = out.cpu().numpy().reshape(nq, ndb)
    got = res[np.array(g["sample_i"]), np.array(g["sample_k"])]
    parity_ok = bool(np.array_equal(got, np.array(g["sqeuclidean_int64"], dtype=np.int64)))

    cpu = None
    if not args.no_cpu:
        import oracle
        cores = cpu_cores()
        rows = np.arange(args.cpu_queries)
        sq = np.concatenate([Qs[qo[i]:qo[i + 1]] for i in rows])
        so = np.concatenate([[0], np.cumsum(np.diff(qo)[rows])]).astype(np.int64)
        t0 = time.perf_counter()
        vals = oracle.dfd_cross_i32(sq, so, DB, dbo, nthreads=cores)
        cw = time.perf_counter() - t0
        s_cells = int(np.sum(np.diff(so))) * int(np.sum(np.diff(dbo)))
        cpu = {"value": s_cells / cw, "unit": "cells/s", "cores": cores, "kind": "oracle",
               "sample": f"first {args.cpu_queries} queries x all 1024 database curves ({s_cells} cells), "
                         f"int64 exact oracle on {cores} threads, {cw:.2f} s",
               "gpu_matches_sample": bool(np.array_equal(vals.reshape(len(rows), ndb), res[rows]))}
    return {
        "value": cells / sec, "ms_per_step": sec * 1e3, "dtype": "f64",
        "config": {"workload": "cross: 1024 queries x 1024 database curves of 256 points, 2-D int32 "
                               "uniform in [-2^15, 2^15), squared Euclidean, int64 results (seed 4)",
                   "npairs": nq * ndb, "cells": cells, "global_batch": nq * ndb},
        "parity": {"exact": True, "sampled_ok": parity_ok, "launch_error_flags": errs},
        "roofline": roofline(info, cells, kms, dim, True), "cpu_baseline": cpu,
    }


def serve_open_loop(srv, queries, rate, nwarm, nmeas, seed=7):
    """Poisson arrivals at `rate`: nwarm requests, then the statistics are
    reset and nmeas more follow; returns the server's statistics of the
    requests completed after the reset (latency from submission to result
    inside the server) and the wall time of the measured part."""
    import queue
    import threading

    import workloads
    total = nwarm + nmeas
    arrivals = workloads.poisson_arrivals(seed=seed, count=total, rate=rate)
    pend = queue.Queue()

    def collect():
        while True:
            item = pend.get()
            if item is None:
                return
            srv.wait(item)

    th = threading.Thread(target=collect)
    gc.collect()
    gc.disable()  # no collector pauses in the client's arrival schedule
    th.start()
    t0 = time.perf_counter()
    tm = None
    for i, ta in enumerate(arrivals):
        if i == nwarm:
            srv.reset_stats()
            tm = time.perf_counter()
        while True:
            dt = t0 + ta - time.perf_counter()
            if dt <= 0:
                break
            time.sleep(min(dt, 0.0005))
        pend.put(srv.submit(queries[i % len(queries)]))
    pend.put(None)
    th.join()
    wall = time.perf_counter() - (tm if tm is not None else t0)
    gc.enable()
    return srv.stats(), wall


def serve_saturation(srv, queries, count):
    """Closed loop: every request submitted at once; requests per second and
    DP cells per second until the last result."""
    srv.reset_stats()
    t0 = time.perf_counter()
    tickets = [srv.submit(queries[i % len(queries)]) for i in range(count)]
    for t in tickets:
        srv.wait(t)
    sec = time.perf_counter() - t0
    return count / sec, srv.stats()


def serving_session(torch, ffd, ctx, dev, slots, nsat, nwarm, nmeas, fractions, qps=0.0):
    """The serving workload: a resident 10,000-curve database, a saturation
    run, then open-loop runs at the given fractions of the saturation rate
    (or at the absolute rate qps)."""
    import workloads
    DB, dbo = workloads.serving_db()
    db_points = int(dbo[-1])
    DBd = torch.from_numpy(DB).to(dev)
    db = ffd.Database(ctx, DBd, dbo)
    srv = ffd.Server(db, max_slots=slots, max_query=8192)
    qs = workloads.serving_queries(count=4096)
    for q in qs[:16]:
        srv.wait(srv.submit(q))
    sat_qps, sat_stats = serve_saturation(srv, qs, nsat)
    print(f"serving: saturation {sat_qps:.0f} requests/s", file=sys.stderr, flush=True)
    runs = []
    rates = [qps] if qps > 0 else [f * sat_qps for f in fractions]
    for k, rate in enumerate(rates):
        st, wall = serve_open_loop(srv, qs, rate, nwarm, nmeas, seed=7 + k)
        runs.append({"qps_target": rate, "fraction_of_saturation": rate / sat_qps, "qps_achieved": st["qps"],
                     "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
                     "max_ms": st["max_ms"], "completed": st["completed"], "failed": st["failed"],
                     "deferred": st["deferred"], "cells_per_s": st["cells_per_s"], "wall_s": wall,
                     "launches_by_rows_per_lane": dict(zip(range(1, 9), st["launches_by_rows"]))})
        print(f"serving: {rate:.0f} requests/s: p50 {st['p50_ms']:.2f} ms, p99 {st['p99_ms']:.2f} ms",
              file=sys.stderr, flush=True)
    info = {"saturation_qps": sat_qps, "saturation_cells_per_s": sat_stats["cells_per_s"],
            "saturation_requests": nsat, "warmup_requests": nwarm, "measured_requests": nmeas,
            "max_slots": slots, "waves": sat_stats["waves"], "requests_per_launch": sat_stats["requests_per_launch"],
            "db_points": db_points, "runs": runs}
    return info, srv, db, DB, dbo, qs


def run_serving(args, torch, ffd, ctx, dev, stream):
    """Queries against the resident 10,000-curve database: a closed-loop
    burst measures the saturation rate S, then Poisson arrivals at 0.25 S,
    0.5 S and 0.8 S (or at --qps) give the latency percentiles and cells/s,
    each over --requests requests after --serving-warmup warm-up ones."""
    import oracle
    import workloads
    fr = [float(x) for x in args.fractions.split(",")]
    info, srv, db, DB, dbo, qs = serving_session(torch, ffd, ctx, dev, args.slots, args.sat_requests,
                                                 args.serving_warmup, args.requests, fr, args.qps)
    # parity of two served results against the oracle
    pick = [0, 1]
    res = [srv.wait(srv.submit(qs[i])).copy() for i in pick]
    sq, so = workloads.concat([qs[i] for i in pick])
    cores = cpu_cores()
    t2 = time.perf_counter()
    want = oracle.dfd_cross(sq, so, DB, dbo, oracle.EUCLIDEAN, nthreads=cores)
    cw = time.perf_counter() - t2
    parity_ok = bool(all(np.all(np.abs(res[r] - want[r]) <= TOL * want[r]) for r in range(len(pick))))
    db_points = info["db_points"]
    s_cells = int(np.sum(np.diff(so))) * db_points
    cpu = None if args.no_cpu else {
        "value": s_cells / cw, "unit": "cells/s", "cores": cores, "kind": "oracle",
        "sample": f"2 queries ({int(np.sum(np.diff(so)))} points) against all 10,000 database curves "
                  f"({s_cells} cells), FP64 rolling-row oracle on {cores} threads, {cw:.2f} s"}
    srv.close()
    db.close()
    head = min(info["runs"], key=lambda r: abs(r["fraction_of_saturation"] - 0.5))
    sat = info["saturation_cells_per_s"]
    launch = {"rows_per_lane": "1 to 8, chosen per request", "waves": info["waves"],
              "requests_per_launch": info["requests_per_launch"]}
    return {
        "value": head["cells_per_s"], "ms_per_step": head["mean_ms"], "dtype": "f32",
        "config": {"workload": "serving: Poisson arrivals, each a query against a resident database of 10,000 "
                               "curves; lengths log-normal (median 300, sigma 1, clipped to [32, 8192]), 2-D "
                               "float32 random walks, Euclidean (seeds 5, 6, 7)",
                   "requests": args.requests, "db_points": db_points, "global_batch": args.requests,
                   "hw_queues": HW_QUEUES},
        "parity": {"tolerance": TOL, "sampled_ok": parity_ok,
                   "failed_requests": sum(r["failed"] for r in info["runs"])},
        "serving": info,
        "roofline": {"bound": "alu", "achieved": sat * imin(2) / 1e12, "peak": PEAK_VALU / 1e12,
                     "unit": "TVALUop/s", "frac": sat * imin(2) / PEAK_VALU, "traffic": None,
                     "kernel": "ffd::stream_kernel<R, 2, float>", "kernel_ms": None, "launch": launch,
                     "basis": "saturation cells/s over the closed-loop burst (host overhead included)"},
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed steps first (the GPU clock ramps up over the first tens of milliseconds)")
    ap.add_argument("--workload", choices=["batched", "plain", "large", "cross", "serving", "dtw", "levenshtein",
                                           "geo", "geo_dtw", "knn", "decide", "short"],
                    default="batched")
    ap.add_argument("--requests", type=int, default=20000, help="measured open-loop requests per rate (serving)")
    ap.add_argument("--serving-warmup", type=int, default=2000, help="open-loop warm-up requests per rate (serving)")
    ap.add_argument("--sat-requests", type=int, default=2000, help="closed-loop burst size (serving)")
    ap.add_argument("--fractions", default="0.25,0.5,0.8",
                    help="open-loop rates as fractions of the saturation rate (serving workload)")
    ap.add_argument("--qps", type=float, default=0.0, help="open-loop arrival rate; 0 = the fractions above")
    ap.add_argument("--no-serving", action="store_true",
                    help="batched workload: skip the serving block (saturation and p50/p99 at half of it)")
    ap.add_argument("--slots", type=int, default=16, help="requests in flight (serving)")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-pair comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-pairs", type=int, default=4096, help="pairs in the CPU oracle sample (batched)")
    ap.add_argument("--cpu-block", type=int, default=32768,
                    help="leading points per curve timed on the CPU (large)")
    ap.add_argument("--cpu-queries", type=int, default=64, help="queries in the CPU oracle sample (cross)")
    ap.add_argument("--knn-batch", type=int, default=64, help="queries per ffd_knn_batch call (knn workload)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 256 MiB device copy (reference for HBM counter scaling)")
    ap.add_argument("--metric", choices=["euclidean", "manhattan", "chebyshev"], default="euclidean",
                    help="ground distance of the batched workload")
    ap.add_argument("--dtw", action="store_true", help="short workload: DTW of squared cells")
    ap.add_argument("--mixed", action="store_true", help="short workload: 800 long pairs among the short ones")
    ap.add_argument("--levenshtein", action="store_true",
                    help="short workload: the Levenshtein distance of short symbol sequences")
    ap.add_argument("--no-short", action="store_true",
                    help="batched workload: skip the short-pairs block (one pair per lane) of the line")
    ap.add_argument("--dim", type=int, default=2,
                    help="coordinates per point of the batched workload (its headline form is 2-D)")
    ap.add_argument("--rows-per-lane", type=int, default=0)
    ap.add_argument("--waves-per-simd", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="time the launch shapes once before the warm-up (batched) and use the fastest")
    ap.add_argument("--split", type=float, default=0.0,
                    help="band splitting: 0 auto, < 0 only when needed, > 0 above this share of a wave's load")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(it measures one GPU's share; batches shard by pairs across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_05708_amd import ffd

    dev = torch.device("cuda:0")
    ctx = ffd.Context(0)
    ctx.set_tuning(args.rows_per_lane, args.waves_per_simd)
    ctx.set_split(args.split)
    stream = torch.cuda.current_stream()
    if args.workload == "batched":
        r = run_batched(args, torch, ffd, ctx, dev, stream)
        if not args.no_serving:
            # the latency half of the metric: p50/p99 at half the saturation rate
            info, srv, db, _, _, _ = serving_session(torch, ffd, ctx, dev, args.slots, args.sat_requests,
                                                     args.serving_warmup, args.requests, [0.5])
            srv.close()
            db.close()
            run = info["runs"][0]
            r["serving"] = {"workload": "10,000-curve resident database, log-normal query lengths (median 300, "
                                        "sigma 1, [32, 8192]), Poisson arrivals at half the saturation rate",
                            "hw_queues": HW_QUEUES,
                            "saturation_qps": info["saturation_qps"],
                            "saturation_cells_per_s": info["saturation_cells_per_s"],
                            "qps": run["qps_achieved"], "p50_ms": run["p50_ms"], "p99_ms": run["p99_ms"],
                            "mean_ms": run["mean_ms"], "cells_per_s": run["cells_per_s"],
                            "requests": run["completed"], "warmup_requests": info["warmup_requests"],
                            "failed": run["failed"]}
        if not args.no_short:
            # many short pairs (one pair per lane) beside the streaming kernel on the same pairs
            import copy
            sa = copy.copy(args)
            sa.steps, sa.warmup, sa.no_cpu, sa.dtw, sa.mixed, sa.levenshtein = 20, 5, True, False, False, False
            sr = run_short(sa, torch, ffd, ctx, dev, stream)
            r["short_pairs"] = {"workload": sr["config"]["workload"], "cells_per_s": sr["value"],
                                "ms_per_step": sr["ms_per_step"], "kernel_ms": sr["roofline"]["kernel_ms"],
                                "frac": sr["roofline"]["frac"], "parity": sr["parity"],
                                "eager_ms_per_step": sr["eager"]["ms_per_step"], "timing": sr["timing"]["timing"],
                                "streaming_kernel_cells_per_s": sr["streaming_kernel"]["cells_per_s"]}
    elif args.workload == "cross":
        r = run_cross(args, torch, ffd, ctx, dev, stream)
    elif args.workload == "serving":
        r = run_serving(args, torch, ffd, ctx, dev, stream)
    elif args.workload == "dtw":
        r = run_dtw(args, torch, ffd, ctx, dev, stream)
    elif args.workload == "levenshtein":
        r = run_levenshtein(args, torch, ffd, ctx, dev, stream)
    elif args.workload in ("geo", "geo_dtw"):
        r = run_geo(args, torch, ffd, ctx, dev, stream, dtw=args.workload == "geo_dtw")
    elif args.workload == "knn":
        r = run_knn(args, torch, ffd, ctx, dev, stream)
    elif args.workload == "decide":
        r = run_decide(args, torch, ffd, ctx, dev, stream)
    elif args.workload == "short":
        r = run_short(args, torch, ffd, ctx, dev, stream)
    else:
        r = run_pair(args, torch, ffd, ctx, dev, stream, args.workload)
    line = {
        "metric": r.get("metric", METRIC), "value": r["value"], "unit": r.get("unit", "cells/s"), "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": r["dtype"], "data": "synthetic",
    }
    for k in ("timing", "eager", "config", "parity", "autotune", "serving", "short_pairs", "search", "roofline",
              "plain", "streaming_kernel", "cpu_baseline"):
        if k in r:
            line[k] = r[k]
    if line.get("cpu_baseline"):
        line["cpu_baseline"].update(cpu_host())
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
