#!/usr/bin/env python3
"""Write the stored expected results of the full-size workloads.

Every value here comes from the CPU oracle (deep MGP, Alg. 1 with the
bipartitioning of Alg. 2 under the deterministic sub-round LP rule) run on the
seeded synthetic generators; nothing is read from the GPU path.

    python tests/golden/make_golden.py [name ...]      # default: all

writes tests/golden/<name>.json with the graph fingerprint (n, m, sha256 of
xadj/adjncy), the partition's sha256 (int32 little-endian), cut, block-weight
digest, per-level sizes and the oracle's counters.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2105_02022_amd import gen  # noqa: E402

# (file name, generator workload, k, eps, seed[, initial-bipartitioning options])
CASES = {
    "grid128_k8": ("grid128", 8, 0.03, 1),
    "rgg20_k64": ("rgg20", 64, 0.03, 1),
    "rmat22_k32768": ("rmat22", 1 << 15, 0.03, 1),
    "rgg20_k64_pool_fm2": ("rgg20", 64, 0.03, 1, {"fm_passes": 2, "ip_pool": 1}),
    "rgg20_k64_ml_fm2": ("rgg20", 64, 0.03, 1, {"fm_passes": 2, "ip_multilevel": 1}),
}


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def graph_fingerprint(g) -> dict:
    return {"n": int(g.n), "m": int(g.m), "maxdeg": int(g.maxdeg),
            "xadj_sha256": sha(np.asarray(g.xadj, np.int32)), "adjncy_sha256": sha(np.asarray(g.adjncy, np.int32))}


def block_weights(part, vwgt, k):
    w = np.ones(len(part), np.int64) if vwgt is None else np.asarray(vwgt, np.int64)
    return np.bincount(part, weights=w, minlength=k).astype(np.int64)


def make(name):
    wl, k, eps, seed = CASES[name][:4]
    opts = CASES[name][4] if len(CASES[name]) > 4 else {}
    t = time.time()
    g = gen.workload(wl)
    t_gen = time.time() - t
    t = time.time()
    r = oracle.partition(g, k, eps, seed, fm_passes=opts.get("fm_passes", 0), pool=bool(opts.get("ip_pool", 0)),
                         adaptive_eps=bool(opts.get("adaptive_eps", 0)),
                         ip_multilevel=bool(opts.get("ip_multilevel", 0)))
    t_or = time.time() - t
    bw = block_weights(r.part, g.vwgt, k)
    out = {
        "workload": wl, "k": k, "eps": eps, "seed": seed, "options": opts, "graph": graph_fingerprint(g),
        "status": r.status, "part_sha256": sha(np.asarray(r.part, np.int32)),
        "block_weights_sha256": sha(bw), "block_weight_max": int(bw.max()), "block_weight_min": int(bw.min()),
        "stats": {kk: (list(map(int, v)) if isinstance(v, list) else int(v)) for kk, v in r.stats.items()},
        "oracle_seconds": round(t_or, 1),
    }
    if k <= 64:
        out["block_weights"] = list(map(int, bw))
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: gen {t_gen:.1f} s, oracle {t_or:.1f} s, cut {r.stats['cut']}", flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(CASES)):
        make(nm)
