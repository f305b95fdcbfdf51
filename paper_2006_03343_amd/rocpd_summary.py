"""Print a short text summary of a rocprofv3 results database (rocpd SQLite).

    python paper_2006_03343_amd/rocpd_summary.py RESULTS.db [--match SUBSTR ...]

Kernel statistics (calls, total and mean duration) and, when the run
collected counters, the mean value per dispatch of each counter for each
kernel.  Kernel names are shortened to the function name.
"""
import argparse
import re
import sqlite3
from collections import defaultdict


def short(name):
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*", "", name)            # drop the argument list
    return name[:110]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--match", nargs="*", default=[])
    a = ap.parse_args()
    con = sqlite3.connect(a.db)
    cur = con.cursor()
    keep = lambda n: not a.match or any(m in n for m in a.match)
    rows = cur.execute("select name, count(*), sum(duration), avg(duration) from kernels "
                       "group by name order by sum(duration) desc").fetchall()
    print(f"{'kernel':110s} {'calls':>6s} {'total_us':>11s} {'mean_us':>10s}")
    for name, n, tot, avg in rows:
        if keep(name):
            print(f"{short(name):110s} {n:6d} {tot / 1e3:11.2f} {avg / 1e3:10.3f}")
    try:
        crow = cur.execute("select kernel_name, counter_name, value from counters_collection").fetchall()
    except sqlite3.Error:
        crow = []
    if crow:
        acc = defaultdict(list)
        for name, cn, val in crow:
            if keep(name):
                acc[(short(name), cn)].append(val)
        print()
        print(f"{'kernel':110s} {'counter':>12s} {'dispatches':>10s} {'mean_per_dispatch':>18s}")
        for (name, cn), v in sorted(acc.items()):
            print(f"{name:110s} {cn:>12s} {len(v):10d} {sum(v) / len(v):18.1f}")


if __name__ == "__main__":
    main()
