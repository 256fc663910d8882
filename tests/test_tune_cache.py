"""The on-disk autotune cache (ffd_set_tune_cache), on the CPU with a
planning-only context: an entry for a request's class changes the launch
shape the planner describes for it (and for any request of the same
class), an entry of zeros keeps the model's choice, other classes and bad
lines are ignored, and explicit tuning settings win over the file."""
import json
import math

import numpy as np
import pytest

from paper_2404_05708_amd import ffd
import workloads


def tune_class(cus, op, D, p_off, q_off, kernel=0, exact=False):
    lg = lambda x: 0 if x < 1 else int(math.floor(math.log2(x) + 0.5))
    na, nb = len(p_off) - 1, len(q_off) - 1
    return (f"gfx950/cu{cus}/op{op}/k{kernel}/{'i32' if exact else 'f32'}/D{D}/L{lg(p_off[-1] / na)}"
            f"/M{lg(q_off[-1] / nb)}/N{lg(na)}/Q{lg(nb)}")


def write(path, entries, junk=()):
    lines = ["{"] + list(junk)
    items = list(entries.items())
    for i, (k, (R, W, S)) in enumerate(items):
        lines.append(f'"{k}": {{"rows_per_lane": {R}, "waves_per_simd": {W}, "split": {S}}}'
                     + ("," if i + 1 < len(items) else ""))
    lines.append("}")
    path.write_text("\n".join(lines) + "\n")


def test_tune_cache_file(tmp_path):
    h = ffd.ffd_create_planner(256, 160 * 1024)
    try:
        P, p_off, Q, q_off = workloads.random_pairs(70, 300, 64, 2048, dim=2)
        auto, _, _ = ffd.ffd_plan_describe(h, ffd.FFD_OP_BATCH, p_off, q_off, 2)
        assert auto["rows_per_lane"] == 8
        key = tune_class(256, ffd.FFD_OP_BATCH, 2, p_off, q_off)
        f = tmp_path / "tune.json"
        write(f, {key: (4, 1, 0.0), "gfx950/cu256/op1/k0/f32/D3/L10/M10/N8/Q8": (2, 2, 0.0)},
              junk=['"broken line', '"x": {"rows_per_lane": 3, "waves_per_simd": 1, "split": 0}'])
        json.loads(f.read_text().replace('"broken line\n', "").replace(
            '"x": {"rows_per_lane": 3, "waves_per_simd": 1, "split": 0}\n', ""))  # the rest is JSON
        ffd.ffd_set_tune_cache(h, str(f))
        sm, _, _ = ffd.ffd_plan_describe(h, ffd.FFD_OP_BATCH, p_off, q_off, 2)
        assert sm["rows_per_lane"] == 4 and sm["waves"] <= 1024
        # another request of the same class (same buckets) takes it too
        P2, p2, Q2, q2 = workloads.random_pairs(71, 300, 64, 2048, dim=2)
        assert tune_class(256, ffd.FFD_OP_BATCH, 2, p2, q2) == key
        assert ffd.ffd_plan_describe(h, ffd.FFD_OP_BATCH, p2, q2, 2)[0]["rows_per_lane"] == 4
        # another class (D = 3) does not
        assert ffd.ffd_plan_describe(h, ffd.FFD_OP_BATCH, p_off, q_off, 3)[0]["rows_per_lane"] == \
            ffd.ffd_plan_describe(ffd.ffd_create_planner(256, 160 * 1024), ffd.FFD_OP_BATCH, p_off, q_off, 3)[0][
                "rows_per_lane"]
        # explicit settings win over the file
        ffd.ffd_set_tuning(h, 2, 0)
        assert ffd.ffd_plan_describe(h, ffd.FFD_OP_BATCH, p_off, q_off, 2)[0]["rows_per_lane"] == 2
        ffd.ffd_set_tuning(h, 0, 0)
        # zeros: the model's choice
        write(f, {key: (0, 0, 0.0)})
        ffd.ffd_set_tune_cache(h, str(f))
        assert ffd.ffd_plan_describe(h, ffd.FFD_OP_BATCH, p_off, q_off, 2)[0]["rows_per_lane"] == 8
        # no file / a missing file: nothing applies
        ffd.ffd_set_tune_cache(h, str(tmp_path / "missing.json"))
        assert ffd.ffd_plan_describe(h, ffd.FFD_OP_BATCH, p_off, q_off, 2)[0]["rows_per_lane"] == 8
        ffd.ffd_set_tune_cache(h, None)
    finally:
        ffd.ffd_destroy(h)
