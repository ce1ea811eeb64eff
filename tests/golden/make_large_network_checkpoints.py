"""Writes the oracle's checkpoints of the 200,000-link network run.

The 200,000-link network (the size of the TIGER network of Section "Graph
partitioning", 2,000,000 vehicles, lane changing with turn lanes and
unprotected priority turns of Section "Microsimulation driving logic") is
stepped by the CPU oracle alone for its whole 7,200-step horizon.  At each
checkpoint the oracle's 12 counters, its state hash and SHA-256 digests of
every per-vehicle state array and of the exit-time array are stored in
large_network_checkpoints.json, which the GPU test compares against.

Only oracle/ and the seeded input generators are used here; nothing comes
from the GPU library.  The run takes about an hour on one core.  With
--snapshot DIR the oracle state at each checkpoint is also saved there, and
--resume restarts from the latest snapshot (a restart from a saved state
equals the uninterrupted run; the oracle's own restart pin covers that), so
an interrupted run loses at most one stretch between checkpoints.

    python tests/golden/make_large_network_checkpoints.py [--snapshot DIR]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_cs_0105004_amd import scenarios as S  # noqa: E402

OUT = os.path.join(HERE, "large_network_checkpoints.json")
CHECKPOINTS = (1800, 3600, 7200)
STAT_KEYS = ("t", "n_waiting", "n_active", "n_arrived", "veh_updates", "sum_v",
             "crossings", "exits", "lane_changes", "insertions", "c_occ",
             "hash")
# counters that sum over steps (a resumed run adds those of the stretch
# before the snapshot)
SUMMED = ("veh_updates", "sum_v", "crossings", "exits", "lane_changes",
          "insertions", "c_occ")
STATE_DTYPES = (("status", np.int8), ("link", np.int32), ("lane", np.int8),
                ("x", np.int32), ("v", np.int8), ("rptr", np.int32),
                ("exit_t", np.int32))


def digests(state: dict) -> dict:
    """SHA-256 of each state array as little-endian bytes of its dtype."""
    out = {}
    for key, dt in STATE_DTYPES:
        a = np.ascontiguousarray(state[key], dtype=np.dtype(dt).newbyteorder("<"))
        out[key] = hashlib.sha256(a.tobytes()).hexdigest()
    return out


def restored(scen, snap: dict):
    """The scenario restarted from a saved oracle state at step snap['t']."""
    return scen.with_state(snap["state"], int(snap["t"]))


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--snapshot", default=None,
                    help="directory for oracle snapshots at each checkpoint")
    ap.add_argument("--resume", action="store_true")
    args = ap.parse_args()
    t_start = time.time()
    scen = S.large_network()
    print(f"generated {scen.name}: {scen.n_links} links, {scen.n_veh} "
          f"vehicles in {time.time() - t_start:.0f} s", flush=True)
    record = {
        "scenario": "large_network(seed=4242): 200,000 directed links, "
                    "2,000,000 vehicles, lane change + turn lanes, 7,200 steps",
        "cite": "lane changing and unprotected turns of Section "
                "'Microsimulation driving logic' on the 200,000-link network "
                "size of Section 'Graph partitioning'; values computed by the "
                "CPU oracle only",
        "writer": "tests/golden/make_large_network_checkpoints.py",
        "checkpoints": [],
    }
    base = {k: 0 for k in SUMMED}
    o = None
    if args.resume and args.snapshot and os.path.exists(OUT):
        with open(OUT) as f:
            record = json.load(f)
        done = [c["stats"]["t"] for c in record["checkpoints"]]
        if done:
            t_last = max(done)
            path = os.path.join(args.snapshot, f"oracle_t{t_last}.npz")
            with np.load(path) as z:
                snap = {"t": int(z["t"]), "state": {k: z[k] for k, _ in STATE_DTYPES}}
            o = oracle.OracleSim(restored(scen, snap))
            last = [c for c in record["checkpoints"] if c["stats"]["t"] == t_last][0]
            base = {k: int(last["stats"][k]) for k in SUMMED}
            print(f"resumed at t={t_last}", flush=True)
    if o is None:
        o = oracle.OracleSim(scen)
    t = o.stats()["t"]
    for cp in CHECKPOINTS:
        if cp <= t:
            continue
        while t < cp:
            k = min(100, cp - t)
            o.step(k)
            t += k
            if t % 600 == 0:
                s = o.stats()
                print(f"t={t} active={s['n_active']} arrived={s['n_arrived']} "
                      f"elapsed={time.time() - t_start:.0f} s", flush=True)
        stats = {k: int(v) for k, v in o.stats().items()}
        for k in SUMMED:
            stats[k] += base[k]
        state = o.state()
        record["checkpoints"].append({"stats": {k: stats[k] for k in STAT_KEYS},
                                      "sha256": digests(state)})
        tmp = OUT + ".tmp"
        with open(tmp, "w") as f:
            json.dump(record, f, indent=1)
            f.write("\n")
        os.replace(tmp, OUT)
        if args.snapshot:
            os.makedirs(args.snapshot, exist_ok=True)
            np.savez(os.path.join(args.snapshot, f"oracle_t{cp}.npz"), t=cp,
                     **{k: state[k] for k, _ in STATE_DTYPES})
        print(f"checkpoint t={cp} written ({time.time() - t_start:.0f} s)",
              flush=True)


if __name__ == "__main__":
    main()
