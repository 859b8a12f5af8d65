"""Summaries of rocprofv3 output databases for the profiles/ folder.

    python -m paper_1702_03154_amd.profsum stats <results.db>          per-kernel durations
    python -m paper_1702_03154_amd.profsum pmc <results.db> <COUNTER>  per-kernel counter values

Kernel names are shortened (namespace and argument list dropped).
"""
from __future__ import annotations

import re
import sqlite3
import sys


def short(name: str) -> str:
    name = name.replace("mphfk::(anonymous namespace)::", "")
    name = re.sub(r"\(.*$", "", name)
    return name[:60]


def stats(db: str, out=sys.stdout):
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), sum(end-start), avg(end-start), min(end-start), "
                     "max(end-start) from kernels group by name order by sum(end-start) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    print(f"{'kernel':60s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>10s} {'min_us':>10s} "
          f"{'max_us':>10s} {'pct':>6s}", file=out)
    for n, k, s, a, lo, hi in rows:
        print(f"{short(n):60s} {k:6d} {s / 1e6:10.3f} {a / 1e3:10.1f} {lo / 1e3:10.1f} {hi / 1e3:10.1f} "
              f"{100 * s / total:6.1f}", file=out)


def pmc(db: str, counter: str, out=sys.stdout):
    c = sqlite3.connect(db)
    cols = [r[1] for r in c.execute("pragma table_info(counters_collection)")]
    name_col = "counter_name" if "counter_name" in cols else "name"
    val_col = "value" if "value" in cols else "counter_value"
    kcol = "kernel_name" if "kernel_name" in cols else "name"
    q = (f"select {kcol}, count(*), avg({val_col}), min({val_col}), max({val_col}) from "
         f"counters_collection where {name_col} = ? group by {kcol} order by avg({val_col}) desc")
    print(f"{'kernel':60s} {'dispatches':>10s} {'avg':>14s} {'min':>14s} {'max':>14s}   ({counter})", file=out)
    for n, k, a, lo, hi in c.execute(q, (counter,)).fetchall():
        print(f"{short(n):60s} {k:10d} {a:14.1f} {lo:14.1f} {hi:14.1f}", file=out)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3])
    else:
        raise SystemExit(__doc__)
