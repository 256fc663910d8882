"""Write the stored expected values under tests/golden/ (oracle only).

Every value here is computed by the CPU oracle (oracle/) on the seeded
synthetic workloads of workloads.py; nothing is read back from the GPU
library.  Re-run after any change to the oracle's arithmetic or to a
generator:

    python tests/golden/make_golden.py [--large]

--large also computes the 131072 x 131072 pair (about a minute of CPU).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_indices(rng, count, total):
    return sorted(set(rng.choice(total, size=min(count, total), replace=False).tolist()))


def main():
    large = "--large" in sys.argv
    nthreads = os.cpu_count() or 1
    out = {"generator": "workloads.py", "oracle": "oracle/ffd_oracle.c (FP64 rolling form)"}

    p, q = workloads.plain_pair()
    out["plain_pair"] = {
        "workload": "plain_pair(seed=1): 512 x 384, 2-D float32 walks",
        "euclidean": oracle.dfd(p, q, oracle.EUCLIDEAN, "table"),
        "sqeuclidean": oracle.dfd(p, q, oracle.SQEUCLIDEAN, "table"),
    }

    P, p_off, Q, q_off = workloads.batched()
    npairs = len(p_off) - 1
    cells = np.diff(p_off) * np.diff(q_off)
    rng = np.random.default_rng(1001)
    idx = sample_indices(rng, 60, npairs)
    idx = sorted(set(idx) | {int(np.argmax(cells)), int(np.argmin(cells))})
    ps, pl = p_off[:-1][idx], np.diff(p_off)[idx]
    qs, ql = q_off[:-1][idx], np.diff(q_off)[idx]
    vals = oracle.dfd_pairs(P, ps, pl, Q, qs, ql, oracle.EUCLIDEAN, nthreads)
    out["batched"] = {
        "workload": "batched(seed=2): 4096 pairs, n, m uniform in [64, 2048], 2-D",
        "total_cells": int(cells.sum()),
        "sample_index": [int(i) for i in idx],
        "euclidean": [float(v) for v in vals],
    }

    # the same pairs under the Manhattan and Chebyshev ground distances
    for name, metric in (("manhattan", oracle.MANHATTAN), ("chebyshev", oracle.CHEBYSHEV)):
        mv = oracle.dfd_pairs(P, ps, pl, Q, qs, ql, metric, nthreads)
        out["batched_" + name] = {
            "workload": f"batched(seed=2) as above, {name} ground distance",
            "sample_index": [int(i) for i in idx],
            name: [float(v) for v in mv],
        }

    # DTW (Appendix B) of squared Euclidean cells on the same pairs
    dvals = oracle.dfd_pairs(P, ps, pl, Q, qs, ql, oracle.SQEUCLIDEAN, nthreads, measure="dtw")
    out["dtw_batched"] = {
        "workload": "batched(seed=2) as above, DTW with squared Euclidean cells",
        "sample_index": [int(i) for i in idx],
        "sqeuclidean": [float(v) for v in dvals],
    }

    # great-circle distances on the sphere workload
    GP, gpo, GQ, gqo = workloads.geo_pairs()
    rng = np.random.default_rng(1004)
    gcells = np.diff(gpo) * np.diff(gqo)
    gidx = sample_indices(rng, 60, len(gpo) - 1)
    gidx = sorted(set(gidx) | {int(np.argmax(gcells)), int(np.argmin(gcells))})
    gv = oracle.dfd_pairs(GP, gpo[:-1][gidx], np.diff(gpo)[gidx], GQ, gqo[:-1][gidx], np.diff(gqo)[gidx],
                          oracle.HAVERSINE, nthreads)
    gd = oracle.dfd_pairs(GP, gpo[:-1][gidx], np.diff(gpo)[gidx], GQ, gqo[:-1][gidx], np.diff(gqo)[gidx],
                          oracle.HAVERSINE, nthreads, measure="dtw")
    out["dtw_haversine"] = {
        "workload": "geo_pairs(seed=9) as below, DTW of great-circle angles (radians)",
        "sample_index": [int(i) for i in gidx],
        "haversine": [float(v) for v in gd],
    }
    out["batched_haversine"] = {
        "workload": "geo_pairs(seed=9): 4096 pairs of (latitude, longitude) walks on the sphere, lengths in "
                    "[64, 2048], great-circle distance (radians)",
        "total_cells": int(gcells.sum()),
        "sample_index": [int(i) for i in gidx],
        "haversine": [float(v) for v in gv],
    }

    # Levenshtein (Appendix B) on the symbol-sequence workload
    SP, spo, SQ, sqo = workloads.symbol_pairs()
    rng = np.random.default_rng(1003)
    sidx = sample_indices(rng, 60, len(spo) - 1)
    lv = oracle.lev_pairs(SP, spo[:-1][sidx], np.diff(spo)[sidx], SQ, sqo[:-1][sidx], np.diff(sqo)[sidx],
                          nthreads)
    out["levenshtein"] = {
        "workload": "symbol_pairs(seed=8): 4096 pairs of 4-letter int32 sequences, lengths in [64, 2048]",
        "sample_index": [int(i) for i in sidx],
        "levenshtein": [int(v) for v in lv],
    }

    Qs, qo, DB, dbo = workloads.cross_int()
    rng = np.random.default_rng(1002)
    ii = rng.integers(0, len(qo) - 1, size=256)
    kk = rng.integers(0, len(dbo) - 1, size=256)
    vals = oracle.dfd_pairs_i32(Qs, qo[ii], qo[ii + 1] - qo[ii], DB, dbo[kk],
                                dbo[kk + 1] - dbo[kk], nthreads)
    out["cross_int"] = {
        "workload": "cross_int(seed=4): 1024 x 1024 curves of 256 points, int32, squared",
        "sample_i": [int(i) for i in ii], "sample_k": [int(k) for k in kk],
        "sqeuclidean_int64": [int(v) for v in vals],
    }

    if large:
        p, q = workloads.large_pair()
        t0 = time.time()
        v = oracle.dfd(p, q, oracle.EUCLIDEAN, "rolling")
        out["large_pair"] = {
            "workload": "large_pair(seed=3): 131072 x 131072, 3-D float32 walks",
            "euclidean": v, "oracle_seconds_single_thread": time.time() - t0,
        }
    else:
        old = os.path.join(HERE, "expected.json")
        if os.path.exists(old):
            prev = json.load(open(old))
            if "large_pair" in prev:
                out["large_pair"] = prev["large_pair"]

    with open(os.path.join(HERE, "expected.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", os.path.join(HERE, "expected.json"))


if __name__ == "__main__":
    main()
