"""Summaries of rocprofv3 output for the step kernels.

    python -m paper_cs_0105004_amd.profiling stats  <run_kernel_stats.csv | run_results.db>
    python -m paper_cs_0105004_amd.profiling pmc    <run_counter_collection.csv | run_results.db> [LAST]
    python -m paper_cs_0105004_amd.profiling copy   <run_counter_collection.csv | run_results.db> BYTES
    python -m paper_cs_0105004_amd.profiling last   <run_kernel_trace.csv> N

`stats` prints calls / average / total duration per kernel from a
`--kernel-trace --stats` run; `pmc` prints, per kernel, the dispatch count and
the mean of every collected counter per dispatch (FETCH_SIZE and WRITE_SIZE
are in KiB), over the LAST dispatches of each kernel if given; `copy` prints
the bytes one plain copy of BYTES bytes reads and writes according to those
counters, i.e. the calibration factor that turns the counters of the step
kernels into HBM bytes; `last` prints, per kernel, the mean duration of its
last N dispatches in a `--kernel-trace` run (one pass of a bench that runs
several configurations).  `stats`, `pmc` and `copy` read rocprofv3's CSV
output or its SQLite database (`run_results.db`, the default output
format); `last` reads the CSV kernel trace.
"""
from __future__ import annotations

import csv
import sqlite3
import sys
from collections import defaultdict


def short_name(name: str) -> str:
    """`void tr::k_back<false>(...)` -> `k_back<false>`."""
    n = name.split("(")[0].strip()
    if n.startswith("void "):
        n = n[5:]
    return n.split("::")[-1]


def kernel_stats(path: str) -> dict:
    out = {}
    if path.endswith(".db"):
        db = sqlite3.connect(path)
        rows = db.execute("select name, count(*), avg(duration), sum(duration),"
                          " min(duration), max(duration) from kernels"
                          " group by name").fetchall()
        for name, n, avg, tot, mn, mx in rows:
            out[short_name(name)] = {"calls": int(n), "avg_ns": float(avg),
                                     "total_ns": float(tot),
                                     "min_ns": float(mn), "max_ns": float(mx)}
        return out
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            out[short_name(row["Name"])] = {
                "calls": int(row["Calls"]),
                "avg_ns": float(row["AverageNs"]),
                "total_ns": float(row["TotalDurationNs"]),
                "min_ns": float(row["MinNs"]),
                "max_ns": float(row["MaxNs"])}
    return out


def counters(path: str, last: int = 0) -> dict:
    """{kernel: {counter: (dispatches, mean per dispatch)}}, over the `last`
    dispatches of each kernel (in dispatch order) when last > 0."""
    vals = defaultdict(lambda: defaultdict(list))
    if path.endswith(".db"):
        db = sqlite3.connect(path)
        for kn, cn, did, v in db.execute(
                "select kernel_name, counter_name, dispatch_id, value"
                " from counters_collection"):
            vals[short_name(kn)][cn].append((int(did), float(v)))
    else:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                vals[short_name(row["Kernel_Name"])][row["Counter_Name"]].append(
                    (int(row["Dispatch_Id"]), float(row["Counter_Value"])))
    out = {}
    for k, cs in vals.items():
        out[k] = {}
        for c, v in cs.items():
            v.sort()
            if last > 0:
                v = v[-last:]
            out[k][c] = (len(v), sum(x for _, x in v) / max(len(v), 1))
    return out


def last_durations(path: str, n: int) -> dict:
    """{kernel: (dispatches used, mean ns)} over the last n dispatches of
    each kernel, in dispatch order."""
    rows = defaultdict(list)
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            rows[short_name(row["Kernel_Name"])].append(
                (int(row["Dispatch_Id"]),
                 int(row["End_Timestamp"]) - int(row["Start_Timestamp"])))
    out = {}
    for k, v in rows.items():
        v.sort()
        v = v[-n:]
        out[k] = (len(v), sum(d for _, d in v) / max(len(v), 1))
    return out


def main(argv) -> int:
    if len(argv) < 2:
        print(__doc__)
        return 2
    mode, path = argv[0], argv[1]
    if mode == "stats":
        st = kernel_stats(path)
        print(f"{'kernel':36s} {'calls':>8s} {'avg_us':>9s} {'min_us':>8s} "
              f"{'max_us':>8s} {'total_ms':>9s}")
        for k, v in sorted(st.items(), key=lambda kv: -kv[1]["total_ns"]):
            print(f"{k:36s} {v['calls']:8d} {v['avg_ns'] / 1e3:9.3f} "
                  f"{v['min_ns'] / 1e3:8.3f} {v['max_ns'] / 1e3:8.3f} "
                  f"{v['total_ns'] / 1e6:9.3f}")
    elif mode == "pmc":
        last = int(argv[2]) if len(argv) > 2 else 0
        for k, cs in sorted(counters(path, last).items()):
            for c, (n, m) in sorted(cs.items()):
                print(f"{k:36s} {c:14s} dispatches {n:7d} mean {m:14.1f}")
    elif mode == "last":
        n = int(argv[2])
        print(f"{'kernel':36s} {'last':>8s} {'avg_us':>9s}")
        for k, (m, avg) in sorted(last_durations(path, n).items(),
                                  key=lambda kv: -kv[1][1] * kv[1][0]):
            print(f"{k:36s} {m:8d} {avg / 1e3:9.3f}")
    elif mode == "copy":
        nbytes = float(argv[2])
        for k, cs in sorted(counters(path).items()):
            if "copy" not in k.lower():
                continue
            for c, (n, m) in sorted(cs.items()):
                kib = nbytes / 1024.0
                print(f"{k:36s} {c:14s} dispatches {n:4d} mean {m:14.1f} KiB "
                      f"(copy of {kib:.0f} KiB: factor {kib / m:.4f})")
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
