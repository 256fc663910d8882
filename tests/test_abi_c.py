"""The C ABI from C: tests/abi_check.c is compiled with gcc against
include/ffd.h alone and linked with libffd.so (CPU only, a planning-only
context).  Struct sizes and field offsets must match the ctypes mirror in
the Python binding, and the plan the C program reads must be the one the
binding reads for the same request."""
import ctypes
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2404_05708_amd import ffd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.dirname(ffd.LIB_PATH)


@pytest.fixture(scope="module")
def c_output(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path_factory.mktemp("abi") / "abi_check")
    libname = os.path.basename(ffd.LIB_PATH)
    assert libname.startswith("lib") and libname.endswith(".so")
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "abi_check.c"), "-o", exe, "-L", LIBDIR,
                    "-l" + libname[3:-3], "-Wl,-rpath," + LIBDIR], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=120).stdout
    return [json.loads(line) for line in out.splitlines() if line.strip()]


MIRRORS = {"ffd_plan_summary": ffd.PlanSummary, "ffd_plan_job": ffd.PLAN_JOB, "ffd_launch_info": ffd.LaunchInfo,
           "ffd_tuning": ffd.Tuning, "ffd_search_info": ffd.SearchInfo, "ffd_server_stats": ffd.ServerStats}


def layout(mirror, field=None):
    """(size) of a mirror, or (offset, size) of one of its fields: ctypes
    structures, or the numpy record type of the job table"""
    if isinstance(mirror, np.dtype):
        if field is None:
            return mirror.itemsize
        dt, off = mirror.fields[field][:2]
        return off, dt.itemsize
    if field is None:
        return ctypes.sizeof(mirror)
    f = getattr(mirror, field)
    return f.offset, f.size


def test_struct_layouts_match_the_binding(c_output):
    seen = set()
    for rec in c_output:
        if "struct" not in rec:
            continue
        mirror = MIRRORS[rec["struct"]]
        seen.add(rec["struct"])
        if "sizeof" in rec:
            assert layout(mirror) == rec["sizeof"], rec
        else:
            assert layout(mirror, rec["field"]) == (rec["offset"], rec["size"]), rec
    assert seen == set(MIRRORS)


def test_plan_through_c_matches_the_binding(c_output):
    plan = next(r["plan"] for r in c_output if "plan" in r)
    p_off = np.concatenate([[0], np.cumsum([100 + 37 * k for k in range(40)])]).astype(np.int64)
    q_off = np.concatenate([[0], np.cumsum([2000 - 41 * k for k in range(40)])]).astype(np.int64)
    h = ffd.ffd_create_planner(256, 160 * 1024)
    try:
        sm, jobs, wj = ffd.ffd_plan_describe(h, ffd.FFD_OP_BATCH, p_off, q_off, 2)
    finally:
        ffd.ffd_destroy(h)
    for k, v in plan.items():
        if k == "last_wave_jobs":
            assert v == int(wj[-1]) == sm["jobs"]
        else:
            assert sm[k] == v, (k, sm[k], v)


def test_status_codes_through_c(c_output):
    text = next(r["strerror"] for r in c_output if "strerror" in r)
    assert text == ffd.lib.ffd_strerror(ffd.FFD_E_NOMEM).decode()
    assert next(r["bad_tuning_status"] for r in c_output if "bad_tuning_status" in r) == ffd.FFD_E_INVALID
    t = next(r for r in c_output if "timing_on_status" in r)
    assert t == {"timing_on_status": ffd.FFD_E_INVALID, "kernel_time_status": ffd.FFD_OK, "ms": 0.0, "launches": 0}
