"""Summaries of rocprofv3 output (kernel dispatch statistics, PMC counters).

    python -m paper_2105_02022_amd.profsum stats <run_results.db> [top]
    python -m paper_2105_02022_amd.profsum pmc <counter_collection.csv>...

`stats` reads the rocpd SQLite database written by
``rocprofv3 --kernel-trace --stats`` and prints per-kernel launch counts and
durations.  `pmc` sums counters per kernel over the given
``--pmc ... -f csv`` runs (FETCH_SIZE / WRITE_SIZE are in KiB per dispatch).
"""
import collections
import csv
import re
import sqlite3
import sys


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


if __name__ == "__main__":
    if len(sys.argv) < 3:
        print(__doc__)
        sys.exit(1)
    if sys.argv[1] == "stats":
        print_stats(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25)
    else:
        print_pmc(sys.argv[2:])
