"""Sanitizers on the host code (CPU only).  The C oracle, built with
AddressSanitizer and UndefinedBehaviorSanitizer, runs every form on ragged
inputs (tests/sanitize_oracle.c); and the C program that drives the
library's planner through the ABI (tests/abi_check.c) runs against host
objects of the library built with both sanitizers (the device code is the
regular build).  Any report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


@pytest.fixture(scope="module")
def gcc():
    g = shutil.which("gcc")
    if g is None:
        pytest.skip("gcc not found")
    return g


def test_oracle_under_sanitizers(gcc, tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    subprocess.run([gcc, "-std=c11", "-O1", "-ffp-contract=off", *SAN, "-o", exe,
                    os.path.join(ROOT, "oracle", "ffd_oracle.c"), os.path.join(ROOT, "tests", "sanitize_oracle.c"),
                    "-lm", "-lpthread"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.startswith("ok "), r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_planner_under_sanitizers(tmp_path):
    """The host sources of the library (planner, serving, search drivers)
    compiled with both sanitizers, linked with the regular kernel objects of
    the in-tree build, driven by tests/sanitize_planner.c through the C ABI
    on a planning-only context (no GPU).  The HIP runtime's own allocations
    are not leak-checked."""
    import glob
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    clang = "/opt/rocm/llvm/bin/clang"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("hipcc / clang not found")
    from paper_2404_05708_amd import build as B
    kernels = [os.path.join(B.BUILD, n) for n in
               ("ffd_kernels.hip.o", "ffd_kernels_rings.hip.o", "ffd_kernels_pipe.hip.o", "ffd_kernels_serve.hip.o",
                "ffd_bounded.hip.o", "ffd_lanes.hip.o", "ffd_noalloc.hip.o")]
    kernels += sorted(glob.glob(os.path.join(B.BUILD, "ffd_kernels_op.hip_FFD_OP*.o")))
    if not all(os.path.exists(k) for k in kernels):
        pytest.skip("kernel objects are missing from _build: compile the library first")
    csrc = os.path.join(ROOT, "paper_2404_05708_amd", "csrc")
    host_flags = [f for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer")
                  for f in ("-Xarch_host", flag)]
    procs, objs = [], []
    for src in ("ffd_host.cpp", "ffd_server.cpp", "ffd_search.cpp"):
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        cmd = [hipcc, "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off", f"--offload-arch={B.ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_flags,
               "-I", os.path.join(ROOT, "include"), "-I", csrc, "-x", "hip", "-c", os.path.join(csrc, src), "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for pr in procs:
        out, _ = pr.communicate(timeout=600)
        assert pr.returncode == 0, out[-3000:]
    drv = str(tmp_path / "sanitize_planner.o")
    subprocess.run([clang, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "sanitize_planner.c"),
                    "-o", drv], check=True)
    exe = str(tmp_path / "sanitize_planner")
    subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                    "-fsanitize=undefined", "-o", exe, drv, *objs, *kernels], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env, cwd=str(tmp_path))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok"), r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
