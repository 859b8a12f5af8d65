"""Summaries of rocprofv3 output databases for the profiles/ folder.

    python -m paper_1702_03154_amd.profsum stats <results.db>          per-kernel durations
    python -m paper_1702_03154_amd.profsum pmc <results.db> <COUNTER>  per-kernel counter values
    python -m paper_1702_03154_amd.profsum traffic <fetch.db> <write.db> <kernel> <queries> <out.json>
        HBM bytes of one launch of <kernel>, each counter scaled by what it reads for the
        1 GiB calibration copy (bench.py --calibrate-copy) run in the same process
    python -m paper_1702_03154_amd.profsum build-traffic <fetch.db> <write.db> <keys> <out.json>
        the same for every library kernel of the one build before the first lookup
    python -m paper_1702_03154_amd.profsum steps <results.db> <k>
        the first k build + lookup steps of a kernel trace, one line each: the summed durations of
        the library kernels from the step's first kernel to its k_lookup (the build's kernel time),
        the span of those kernels on the device clock, and the k_lookup launch itself

Kernel names are shortened (namespace and argument list dropped).
"""
from __future__ import annotations

import re
import sqlite3
import sys


def short(name: str) -> str:
    name = name.replace("mphfk::", "").replace("(anonymous namespace)::", "")
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


SOURCES = ("kernels.hip", "device.h", "internal.h")   # the lookup kernel and the device code it inlines
BUILD_SOURCES = ("kernels.hip", "partition.hip", "device.h", "internal.h", "api.hip")   # the build


def source_digest(sources=SOURCES) -> str:
    """SHA-256 over the sources a kernel (by default the lookup kernel) is built from."""
    import hashlib
    import os
    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in sources:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _per_dispatch(db: str, counter: str):
    c = sqlite3.connect(db)
    return c.execute("select dispatch_id, kernel_name, value from counters_collection "
                     "where counter_name = ? order by dispatch_id", (counter,)).fetchall()


def _calibration(rows):
    """The 1 GiB calibration copy: the largest runtime copy kernel before the first library kernel
    (the library's own small host-to-device copies also run as copy kernels)."""
    first = next(i for i, r in enumerate(rows) if "mphfk" in r[1])
    cal = [r for r in rows[:first] if "copyBuffer" in r[1]]
    return max(r[2] for r in cal)


def traffic(fetch_db: str, write_db: str, kernel: str, queries: int, out_json: str):
    import hashlib
    import json
    import os
    f_rows = _per_dispatch(fetch_db, "FETCH_SIZE")
    w_rows = _per_dispatch(write_db, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    fs = gib_kib / _calibration(f_rows)
    ws = gib_kib / _calibration(w_rows)
    fk = [r[2] for r in f_rows if short(r[1]) == kernel]
    wk = [r[2] for r in w_rows if short(r[1]) == kernel]
    res = {"kernel": kernel, "queries": queries,
           "fetch_kib": sum(fk) / len(fk), "write_kib": sum(wk) / len(wk),
           "fetch_scale": fs, "write_scale": ws,
           "bytes_per_launch": (sum(fk) / len(fk) * fs + sum(wk) / len(wk) * ws) * 1024.0,
           "source_sha256": source_digest()}
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


def build_traffic(fetch_db: str, write_db: str, keys: int, out_json: str):
    """HBM bytes of one build: every library kernel dispatched before the first lookup, each counter
    scaled by the calibration copy."""
    import json
    f_rows = _per_dispatch(fetch_db, "FETCH_SIZE")
    w_rows = _per_dispatch(write_db, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    fs = gib_kib / _calibration(f_rows)
    ws = gib_kib / _calibration(w_rows)

    def build_kib(rows):
        end = next(r[0] for r in rows if short(r[1]) == "k_lookup")
        return sum(r[2] for r in rows if "mphfk" in r[1] and r[0] < end)

    fk, wk = build_kib(f_rows), build_kib(w_rows)
    res = {"what": "one plain build", "keys": keys, "fetch_kib": fk, "write_kib": wk,
           "fetch_scale": fs, "write_scale": ws, "bytes_per_build": (fk * fs + wk * ws) * 1024.0,
           "source_sha256": source_digest(BUILD_SOURCES)}
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")
    print(json.dumps(res, indent=1))


def _is_library(name: str) -> bool:
    """A kernel of the build or lookup path (the roofline probes are left out)."""
    sn = short(name)
    return ("mphfk" in name or sn.startswith(("k_", "void k_"))) and "k_probe" not in sn


def steps(db: str, k: int, out=sys.stdout):
    """Splits a kernel trace of bench.py into its build + lookup steps: each step ends with a
    k_lookup dispatch, and its build is every library kernel dispatched since the previous one."""
    c = sqlite3.connect(db)
    rows = c.execute("select name, start, end, grid_x, workgroup_x from kernels order by start").fetchall()
    print(f"{'step':>4s} {'build_kernels':>14s} {'build_kernel_ms':>16s} {'build_span_ms':>14s} "
          f"{'lookup_ms':>10s} {'lookup_grid':>12s} {'lookup_wg':>10s}", file=out)
    cur, done, lk, last = [], 0, [], []
    for name, t0, t1, gx, wx in rows:
        if not _is_library(name):
            continue
        if short(name) == "k_lookup":
            busy = sum(b - a for _, a, b in cur)
            span = (cur[-1][2] - cur[0][1]) if cur else 0
            print(f"{done:4d} {len(cur):14d} {busy / 1e6:16.3f} {span / 1e6:14.3f} {(t1 - t0) / 1e6:10.3f} "
                  f"{gx:12d} {wx:10d}", file=out)
            lk.append((t1 - t0) / 1e6)
            last = cur
            cur = []
            done += 1
            if done == k:
                break
        else:
            cur.append((short(name), t0, t1))
    if len(lk) > 1:
        print(f"mean k_lookup over steps 1..{len(lk) - 1} (after the first): "
              f"{sum(lk[1:]) / (len(lk) - 1):.3f} ms", file=out)
    if last:
        # the build of the last step by kernel, in order of first dispatch
        agg = {}
        for n, a, b in last:
            c, t, big = agg.get(n, (0, 0, 0))
            agg[n] = (c + 1, t + (b - a), max(big, b - a))
        print(f"\nbuild of step {done - 1} by kernel:", file=out)
        print(f"{'kernel':48s} {'calls':>6s} {'total_ms':>9s} {'longest_ms':>11s}", file=out)
        for n, (c, t, big) in agg.items():
            print(f"{n:48s} {c:6d} {t / 1e6:9.3f} {big / 1e6:11.3f}", file=out)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(float(sys.argv[5])), sys.argv[6])
    elif sys.argv[1] == "steps":
        steps(sys.argv[2], int(sys.argv[3]))
    elif sys.argv[1] == "build-traffic":
        build_traffic(sys.argv[2], sys.argv[3], int(float(sys.argv[4])), sys.argv[5])
    else:
        raise SystemExit(__doc__)
