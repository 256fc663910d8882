"""Schedule simulator for the library's launch plans (CPU, test helper).

Replays a plan (from ffd_plan_describe) the way the kernel walks it: each
wave runs its jobs in order; a job runs its column curves in order and, for
each, its bands in order; a task lasts task_len(m) stream steps (at least
16 separators and m columns, at least 80, a multiple of 16), an idle job
its step count.  From that replay it checks, without a GPU, the properties the
kernel relies on:

* every (row curve, column curve) pair runs each of its bands exactly once,
  and every output index is written exactly once, by the last band;
* a band whose row above comes from the same wave (hand-off) directly
  follows the band above in that wave's stream;
* a band whose row above comes over a global link reads the buffer and flag
  the band above writes, with the same column-curve sequence, and starts at
  least 320 stream steps after it (so every wait is for a strictly earlier
  stream position: no deadlock); a band fed through an LDS ring reads the
  ring of a wave of its own workgroup and starts at least 80 steps after
  the band above;
* link buffers lie inside the plan's link area and flags inside its flag
  count; no two links share a flag unless they are the in-place chain of
  one unit on one wave;
* the longest stream equals the plan's stream_steps.
"""
from collections import defaultdict

import numpy as np

KWAVE, KGROUP, KMIN = 64, 16, 80
LINK_LAG = 320
RING_LAG = KWAVE + KGROUP
ROW_IDLE = 2


def task_len(m):
    # at least 16 separator columns, then the m columns, in whole groups
    return max((m + 2 * KGROUP - 1) // KGROUP * KGROUP, KMIN)


def curve_len(offs, sel, idx):
    o = offs[sel]
    return int(o[idx + 1] - o[idx])


def replay(summary, jobs, wave_jobs, offs):
    """Tasks of every wave: dicts with wave, S, L, row, col, band, nb, hin,
    hout, links and flags."""
    R = summary["rows_per_lane"]
    tasks = []
    ends = []
    for w in range(summary["waves"]):
        S = 0
        for j in range(wave_jobs[w], wave_jobs[w + 1]):
            jb = jobs[j]
            if jb["row_sel"] == ROW_IDLE:
                S += int(jb["col_count"])
                continue
            n = curve_len(offs, jb["row_sel"], jb["row_idx"])
            nb = (n + KWAVE * R - 1) // (KWAVE * R)
            bf = int(jb["band_first"])
            bc = int(jb["band_count"])
            be = min(bf + bc, nb) if bc > 0 else nb
            rel = 0
            for c in range(int(jb["col_count"])):
                col = int(jb["col_first"]) + c
                m = curve_len(offs, jb["col_sel"], col)
                L = task_len(m)
                for b in range(bf, be):
                    if b == 0:
                        hin = "ghost"
                    elif b == bf:
                        hin = "ring" if jb["flag_in"] <= -2 else "link"
                    else:
                        hin = "hand"
                    if b == nb - 1:
                        hout = "sink"
                    elif b + 1 == be:
                        hout = "ring" if jb["flag_out"] == -2 else "link"
                    else:
                        hout = "hand"
                    tasks.append(dict(
                        wave=w, S=S, L=L, row=(int(jb["row_sel"]), int(jb["row_idx"])),
                        col=(int(jb["col_sel"]), col), ci=c, band=b, nb=nb, hin=hin, hout=hout,
                        link_in=int(jb["link_in"]) + rel, link_out=int(jb["link_out"]) + rel,
                        flag_in=int(jb["flag_in"]), flag_out=int(jb["flag_out"]),
                        out=int(jb["out_base"]) + c * int(jb["out_stride"]) if b == nb - 1 else None,
                        job=j))
                    S += L
                rel += L
        ends.append(S)
    return tasks, ends


def check(summary, jobs, wave_jobs, offs, expected_outputs):
    """Assert the plan properties listed in the module docstring."""
    tasks, ends = replay(summary, jobs, wave_jobs, offs)
    assert len(wave_jobs) == summary["waves"] + 1 and wave_jobs[0] == 0 and wave_jobs[-1] == len(jobs)
    assert max(ends) == summary["stream_steps"], (max(ends), summary["stream_steps"])

    by_key = defaultdict(dict)
    outs = defaultdict(int)
    for t in tasks:
        key = (t["row"], t["col"])
        assert t["band"] not in by_key[key], ("band twice", key, t["band"])
        by_key[key][t["band"]] = t
        if t["out"] is not None:
            outs[t["out"]] += 1
    for key, bands in by_key.items():
        nb = next(iter(bands.values()))["nb"]
        assert sorted(bands) == list(range(nb)), ("bands missing", key, sorted(bands), nb)
    assert dict(outs) == {o: 1 for o in expected_outputs}, "outputs not written exactly once"

    wpb = summary["waves_per_block"]
    flag_users = defaultdict(set)
    for key, bands in by_key.items():
        for b, t in bands.items():
            if b == 0:
                assert t["hin"] == "ghost"
                continue
            up = bands[b - 1]
            if t["hin"] == "hand":
                assert up["wave"] == t["wave"] and up["S"] + up["L"] == t["S"], ("hand-off not adjacent", key, b)
                assert up["hout"] == "hand"
            elif t["hin"] == "link":
                assert up["hout"] == "link", ("link without producer", key, b)
                assert up["link_out"] == t["link_in"] and up["flag_out"] == t["flag_in"] >= 0
                assert t["S"] >= up["S"] + LINK_LAG, ("link lag", key, b, up["S"], t["S"])
                assert 0 <= t["link_in"] and t["link_in"] + t["L"] <= summary["link_elems"]
                assert t["flag_in"] < summary["flags"]
                pj, cj = jobs[up["job"]], jobs[t["job"]]
                assert (pj["col_sel"], pj["col_first"], pj["col_count"]) == \
                    (cj["col_sel"], cj["col_first"], cj["col_count"]), "link rows differ in column curves"
                flag_users[t["flag_in"]].add((up["job"], t["job"]))
            else:
                assert t["hin"] == "ring" and up["hout"] == "ring"
                src = -2 - t["flag_in"]
                assert src == up["wave"] % wpb and up["wave"] // wpb == t["wave"] // wpb, ("ring across blocks",
                                                                                           key, b)
                assert t["S"] >= up["S"] + RING_LAG, ("ring lag", key, b, up["S"], t["S"])
    for flag, users in flag_users.items():
        assert len(users) == 1, ("flag shared by two links", flag, users)
    return tasks
