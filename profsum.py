"""Summaries of rocprofv3 output (kernel dispatch statistics, PMC counters).

    python profsum.py stats <run_results.db> [top]
    python profsum.py pmc <counter_collection.csv>...
    python profsum.py copy <MiB> [reps]
    python profsum.py traffic <fetch.csv> <write.csv> <copy_fetch.csv> <copy_write.csv> <MiB>

`stats` reads the rocpd SQLite database written by
``rocprofv3 --kernel-trace --stats`` and prints per-kernel launch counts and
durations.  `pmc` sums counters per kernel over the given
``--pmc ... -f csv`` runs (FETCH_SIZE / WRITE_SIZE are in KiB per dispatch).
`copy` runs a plain device-to-device copy of a known size (the calibration
kernel for the HBM counters).  `traffic` turns a FETCH_SIZE run and a
WRITE_SIZE run of the benchmark into HBM bytes per launch for every kernel
family, each scaled by what the same counter reads for the calibration copy
(expected bytes / counted bytes), and prints a markdown summary that ends in
a JSON block keyed by kernel family (the benchmark reads that block).
"""
import collections
import csv
import re
import sqlite3
import sys


import hashlib
import json
import os


def source_hash() -> str:
    """Digest of the HIP sources, so a stored counter summary is used only for the kernels it measured."""
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2105_02022_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def family(name: str) -> str:
    """Kernel family: the short name without namespace, return type and template arguments."""
    s = short_name(name)
    s = re.sub(r"^void\s+", "", s)
    s = re.sub(r"^kmp::", "", s)
    return re.sub(r"<.*$", "", s)


def short_name(name: str) -> str:
    s = re.sub(r"\(anonymous namespace\)::", "", name)
    return re.sub(r"\((?!anon).*$", "", s)


def kernel_stats(db_path: str):
    con = sqlite3.connect(db_path)
    cur = con.cursor()
    rows = cur.execute("select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
                       "from kernels group by name order by sum(duration) desc").fetchall()
    return [(short_name(r[0]), r[1], r[2], r[3], r[4], r[5]) for r in rows]


def print_stats(db_path: str, top: int = 25):
    rows = kernel_stats(db_path)
    tot = sum(r[2] for r in rows)
    print(f"total kernel time {tot / 1e6:.3f} ms over {sum(r[1] for r in rows)} dispatches")
    print(f"{'total_ms':>10} {'share':>6} {'launches':>9} {'avg_us':>10} {'min_us':>9} {'max_us':>9}  kernel")
    for name, cnt, s, avg, mn, mx in rows[:top]:
        print(f"{s / 1e6:10.3f} {100 * s / tot:5.1f}% {cnt:9d} {avg / 1e3:10.2f} {mn / 1e3:9.2f} {mx / 1e3:9.2f}  {name}")


def pmc(paths):
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for p in paths:
        for r in csv.DictReader(open(p)):
            k = short_name(r["Kernel_Name"])
            agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[(k, r["Counter_Name"])].add(r["Dispatch_Id"])
    return agg, disp


def print_pmc(paths):
    agg, disp = pmc(paths)
    for k, d in sorted(agg.items()):
        print(k)
        for c, v in sorted(d.items()):
            n = len(disp[(k, c)])
            print(f"    {c:24s} total {v:16.0f}  dispatches {n:6d}  per dispatch {v / max(n, 1):14.1f}")


def copy_kernel(mib: int, reps: int = 3):
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}", flush=True)


def _per_dispatch(path, counter, fam_filter=None):
    """{family: (sum of counter over dispatches, dispatch count)} for one csv."""
    tot = collections.defaultdict(float)
    ids = collections.defaultdict(set)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        f = family(r["Kernel_Name"])
        if fam_filter and not fam_filter(f):
            continue
        tot[f] += float(r["Counter_Value"])
        ids[f].add(r["Dispatch_Id"])
    return {f: (tot[f], len(ids[f])) for f in tot}


def traffic(fetch_csv, write_csv, cfetch_csv, cwrite_csv, mib):
    exp_kib = mib * 1024.0
    cf = _per_dispatch(cfetch_csv, "FETCH_SIZE", lambda f: "copy" in f.lower())
    cw = _per_dispatch(cwrite_csv, "WRITE_SIZE", lambda f: "copy" in f.lower())
    (cf_sum, cf_n), = [v for v in cf.values()][:1]
    (cw_sum, cw_n), = [v for v in cw.values()][:1]
    f_scale = exp_kib / (cf_sum / cf_n)
    w_scale = exp_kib / (cw_sum / cw_n)
    fe = _per_dispatch(fetch_csv, "FETCH_SIZE")
    wr = _per_dispatch(write_csv, "WRITE_SIZE")
    out = {"source_hash": source_hash(), "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
           "calibration": f"device copy of {mib} MiB: FETCH_SIZE {cf_sum / cf_n:.0f} KiB, "
                          f"WRITE_SIZE {cw_sum / cw_n:.0f} KiB per dispatch", "kernels": {}}
    print(f"calibration: {out['calibration']} (expected {exp_kib:.0f} KiB each); "
          f"scales fetch {f_scale:.4f}, write {w_scale:.4f}\n")
    print(f"| kernel family | dispatches | FETCH KiB/launch | WRITE KiB/launch | HBM bytes/launch (scaled) |")
    print("|---|---|---|---|---|")
    for f in sorted(set(fe) & set(wr), key=lambda f: -(fe[f][0] + wr[f][0])):
        fk = fe[f][0] / fe[f][1]
        wk = wr[f][0] / wr[f][1]
        b = (fk * f_scale + wk * w_scale) * 1024.0
        out["kernels"][f] = {"dispatches": fe[f][1], "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                             "hbm_bytes_per_launch": round(b)}
        print(f"| {f} | {fe[f][1]} | {fk:.1f} | {wk:.1f} | {b:.0f} |")
    print("\n```json")
    print(json.dumps(out, indent=1))
    print("```")


if __name__ == "__main__":
    if len(sys.argv) < 3:
        print(__doc__)
        sys.exit(1)
    if sys.argv[1] == "stats":
        print_stats(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25)
    elif sys.argv[1] == "copy":
        copy_kernel(int(sys.argv[2]), int(sys.argv[3]) if len(sys.argv) > 3 else 3)
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:6], int(sys.argv[6]))
    else:
        print_pmc(sys.argv[2:])
