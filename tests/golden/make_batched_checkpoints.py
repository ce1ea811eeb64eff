"""Writes the oracle's checkpoints of the 64 batched replications.

The batched workload is 64 independent Portland-style grids of 1,000 to
20,000 links (417,006 links and 4.1M vehicles in all), each with its own
Philox seed, run for 3,600 steps.  Every replication is stepped by the CPU
oracle alone (one process per replication, at most eight at a time); at
t = 1,800 and 3,600 its 12 counters, its state hash and SHA-256 digests of
every per-vehicle state array and of the exit-time array are stored in
batched_checkpoints.json, which the GPU test of the batched step compares
against.  Only oracle/ and the seeded input generators are used here.

    python tests/golden/make_batched_checkpoints.py
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_cs_0105004_amd import scenarios as S  # noqa: E402

OUT = os.path.join(HERE, "batched_checkpoints.json")
CHECKPOINTS = (1800, 3600)
STAT_KEYS = ("t", "n_waiting", "n_active", "n_arrived", "veh_updates", "sum_v",
             "crossings", "exits", "lane_changes", "insertions", "c_occ",
             "hash")
STATE_DTYPES = (("status", np.int8), ("link", np.int32), ("lane", np.int8),
                ("x", np.int32), ("v", np.int8), ("rptr", np.int32),
                ("exit_t", np.int32))

_SCENS = None  # the replications, shared with the worker processes by fork


def digests(state: dict) -> dict:
    """SHA-256 of each state array as little-endian bytes of its dtype."""
    out = {}
    for key, dt in STATE_DTYPES:
        a = np.ascontiguousarray(state[key], dtype=np.dtype(dt).newbyteorder("<"))
        out[key] = hashlib.sha256(a.tobytes()).hexdigest()
    return out


def run_one(k: int) -> dict:
    sc = _SCENS[k]
    o = oracle.OracleSim(sc)
    cps, t = [], 0
    for cp in CHECKPOINTS:
        o.step(cp - t)
        t = cp
        st = o.stats()
        cps.append({"stats": {key: int(st[key]) for key in STAT_KEYS},
                    "sha256": digests(o.state())})
    o.close()
    return {"replication": k, "links": int(sc.n_links),
            "vehicles": int(sc.n_veh), "checkpoints": cps}


def main() -> None:
    global _SCENS
    t0 = time.time()
    _SCENS = S.batched_scenarios()
    print(f"generated {len(_SCENS)} replications in {time.time() - t0:.0f} s",
          flush=True)
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        reps = pool.map(run_one, range(len(_SCENS)), chunksize=1)
    record = {
        "scenario": "batched_scenarios(n=64, seed=77): 64 Portland-style "
                    "grids of 1k-20k links, 5-15 vehicles per link, 3,600 "
                    "steps, Philox seed 1000 + k",
        "cite": "the car following, intersections and parking of Section "
                "'Microsimulation driving logic' on independent replications "
                "(the series of runs of Section 'Adaptive Load Balancing'); "
                "values computed by the CPU oracle only",
        "writer": "tests/golden/make_batched_checkpoints.py",
        "replications": reps,
    }
    with open(OUT, "w") as f:
        json.dump(record, f, indent=1)
        f.write("\n")
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
