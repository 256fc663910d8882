"""Build the HIP library (libffd.so) for gfx950 with hipcc, in-tree.

Flags: -O3; no floating-point contraction (every multiply and add in the
distance is the operation written in the source); denormals kept; packed
FP32 instructions disabled for the device code.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libffd.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
# (source, preprocessor definitions): ffd_kernels_op.hip is compiled once
# per measure / ground distance (OP = measure + 2 * cell)
SOURCES = [("ffd_kernels.hip", {}), ("ffd_kernels_rings.hip", {}), ("ffd_kernels_pipe.hip", {})] + \
          [("ffd_kernels_op.hip", {"FFD_OP": op}) for op in (1, 3, 4, 5, 6, 7, 8, 10, 11)] + \
          [("ffd_kernels_serve.hip", {}), ("ffd_bounded.hip", {}), ("ffd_lanes.hip", {}), ("ffd_noalloc.hip", {}), ("ffd_host.cpp", {}), ("ffd_server.cpp", {}), ("ffd_search.cpp", {})]


# Extra flags per source.  The pipelined single-pair kernel runs one wave per
# SIMD, so nothing hides an instruction's latency but the instruction order:
# the scheduler that maximises instruction-level parallelism suits it
# (measured: 5 % faster on the 131072 x 131072 pair).
EXTRA = {"ffd_kernels_pipe.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}


def _compile(item):
    src, defs = item
    tag = "".join(f"_{k}{v}" for k, v in defs.items())
    obj = os.path.join(BUILD, src + tag + ".o")
    cmd = [HIPCC] + COMMON + EXTRA.get(src, []) + [f"-D{k}={v}" for k, v in defs.items()] + \
        ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {src}")
    return obj


# A debug variant for the stress tests: the streaming kernels pause for a
# pseudo-random time before each progress publication (FFD_DEBUG_JITTER);
# everything else is the release objects.
JITTER_LIB = os.path.join(HERE, "libffd_jitter.so")
JITTER_SOURCES = [("ffd_kernels.hip", {"FFD_DEBUG_JITTER": 1}), ("ffd_kernels_rings.hip", {"FFD_DEBUG_JITTER": 1})]


def _link(objs, lib, verbose):
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(tmp, lib)


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    items = SOURCES + JITTER_SOURCES
    with ThreadPoolExecutor(min(len(items), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, items))
    release, jitter = objs[:len(SOURCES)], objs[len(SOURCES):]
    _link(release, LIB, verbose)
    _link(jitter + release[len(JITTER_SOURCES):], JITTER_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
