#!/usr/bin/env python3
"""Throughput of the TRANSIMS per-second update on one MI355X.

One step = one simulated second of the whole network (parking insertion,
lane-change sub-step, intersections, car following and move) through the
HIP kernels of libtransims, called via its C ABI.  The default workload is
the Portland-sized synthetic network (77 x 78 grid thinned to 20,024
directed links of 1-3 lanes, 200,000 routed vehicles departing uniformly in
the first 1,800 s, vmax 5, p = 0.2), run for its full 3,600-step horizon
from t = 0 with all inputs resident in HBM.

Prints one JSON line with vehicle-updates/s, the simulated-to-real-time
ratio, the roofline position of the dominant kernel (timed with HIP events)
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
METRIC = ("vehicle-updates/sec & sim/real-time ratio (1 GPU, bit-exact); "
          "p50/p99 run latency")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str, steps: int):
    from paper_cs_0105004_amd import scenarios as S
    if name == "portland":
        scen = S.portland_like(T=steps)
        cfg = {"workload": "portland_like_grid", "links": scen.n_links,
               "nodes": scen.n_nodes, "lanes": int(scen.link_lanes.sum()),
               "vehicles": scen.n_veh, "horizon_steps": steps, "vmax": 5,
               "p": 0.2, "lane_change": False}
    elif name == "ring":
        scen = S.ring(T=steps)
        cfg = {"workload": "ring_1000_cells", "vehicles": 150,
               "horizon_steps": steps, "vmax": 5, "p": 0.2}
    else:
        raise SystemExit(f"unknown workload {name}")
    return scen, cfg


# Algorithmic bytes of the method per step (the lattice formulation: every
# cell of an occupied lane read and written once as int8, each active
# vehicle's int32 id read and written, 16 B per crossing or trip end for its
# route entry, exit time and handoff record, 8 B per vehicle leaving parking):
#   B(t) = 2*C_occ(t) + 8*N(t) + 16*X(t) + 8*I(t)
# The move kernel does the first three terms, the front kernel the last.
def algorithmic_bytes(kind, st):
    if kind == "back":
        return (2.0 * st["c_occ"] + 8.0 * st["veh_updates"]
                + 16.0 * (st["crossings"] + st["exits"]))
    if kind == "front":
        return 8.0 * st["insertions"]
    return 2.0 * st["c_occ"] + 8.0 * st["veh_updates"]  # ring: one launch


KERNEL_SOURCES = ("kernels.hip", "kernels.h", "layout.h", "philox.h")


def kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_cs_0105004_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# HBM bytes per launch of the move kernel on the default workload, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over the run)
# scaled by what the same counters read for a plain copy of known size.
# Valid only for the kernel sources with this digest.
MEASURED_TRAFFIC = {
    # FETCH 2860.0 KiB x 2.0 + WRITE 2284.9 KiB x 1.0 per dispatch
    "3de1834b6ced0b63": {"kernel": "back", "steps": 3600,
                         "bytes_per_launch": 8004.3 * 1024},
}


def copy_calibration(nbytes: int, reps: int = 5):
    """Plain device-to-device copies of nbytes bytes, for calibrating the
    memory counters (run under rocprofv3 --pmc)."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)
    return 0


def cpu_baseline(scen, budget_s: float):
    """The oracle on the first steps of the same workload, until about
    budget_s seconds of CPU time have been spent."""
    import oracle
    o = oracle.OracleSim(scen)
    t0 = time.perf_counter()
    steps = 0
    chunk = 25
    while time.perf_counter() - t0 < budget_s and steps < scen.T:
        o.step(min(chunk, scen.T - steps))
        steps += min(chunk, scen.T - steps)
    dt = time.perf_counter() - t0
    st = o.stats()
    return {"value": st["veh_updates"] / dt, "unit": "vehicle-updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"steps 0..{steps - 1} of the same workload "
                      f"({st['veh_updates']} vehicle-updates, {dt:.1f} s, "
                      f"single thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3600)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="portland")
    ap.add_argument("--tile-lanes", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--reps", type=int, default=5,
                    help="further runs of K steps for the run-latency "
                         "percentiles")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    metavar="BYTES", help="only run plain copies of BYTES")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not "
              f"supported (scenarios are independent and would shard by "
              f"slot, see the design notes)", file=sys.stderr)
        return 2

    import torch
    from paper_cs_0105004_amd.sim import Context

    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        return copy_calibration(args.copy_calibration)
    log(f"bench: generating workload {args.workload}")
    scen, cfg = make_workload(args.workload, args.steps)
    ctx = Context(max_slots=2, tile_lanes=args.tile_lanes)

    # warm-up on a throw-away copy, then a fresh load for the timed run
    log(f"bench: warmup {args.warmup} steps")
    ctx.load(1, scen)
    ctx.step(1, args.warmup)
    ctx.stats(1)
    ctx.unload(1)
    ctx.load(0, scen)
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    ctx.step(0, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.stats(0)
    value = st["veh_updates"] / wall

    # run latency: the same K-step run from a fresh load, several times
    runs = [wall]
    for _ in range(max(args.reps, 0)):
        ctx.load(0, scen)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.step(0, args.steps)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t1)
        assert ctx.stats(0)["hash"] == st["hash"], "repeat run diverged"

    # kernel timing pass: the same K steps again, inside HIP graphs with an
    # event between every two kernels on the library's stream
    ctx.load(0, scen)
    ctx.profile(True)
    ctx.step(0, args.steps)
    kt = ctx.kernel_times()
    ctx.profile(False)
    st2 = ctx.stats(0)
    assert st2["hash"] == st["hash"], "timing pass diverged"
    tiling = ctx.tiling(0)
    K = max(args.steps, 1)
    roof = None
    kinds = [k for k in ("front", "back", "ring") if kt[k][0] > 0]
    if kinds:
        dom = max(kinds, key=lambda k: kt[k][1])
        launches = kt[dom][0]
        avg_ms = kt[dom][1] / launches
        bytes_launch = algorithmic_bytes(dom, st) / launches
        achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
        digest = kernel_digest()
        traffic = None
        tr = MEASURED_TRAFFIC.get(digest)
        if tr is not None and args.workload == "portland" and \
                args.steps == tr["steps"] and dom == tr["kernel"]:
            traffic = tr["bytes_per_launch"]
        roof = {"bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": f"k_{dom}", "avg_launch_us": avg_ms * 1e3,
                "algorithmic_bytes_per_launch": bytes_launch,
                "kernel_sources_digest": digest,
                "kernel_ms": {k: kt[k][1] for k in kinds},
                "launches": {k: kt[k][0] for k in kinds}}
    srt = sorted(runs)

    def pct(q):
        return srt[min(len(srt) - 1, int(round(q * (len(srt) - 1))))] * 1e3
    out = {
        "metric": METRIC, "value": value, "unit": "vehicle-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic", "config": cfg,
        "sim_real_time_ratio": args.steps / wall,
        "vehicle_updates": st["veh_updates"], "wall_s": wall,
        "bit_exact_state_hash": f"{st['hash']:016x}",
        "run_latency_ms": {"p50": pct(0.5), "p99": pct(0.99),
                           "runs": len(runs)},
        "tiling": {"tiles": tiling["n_tiles"], "e_dmn": tiling["e_dmn"],
                   "e_tile": tiling["e_tile"]},
        "roofline": roof,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        log(f"bench: oracle sample ({args.cpu_seconds:.0f} s budget)")
        out["cpu_baseline"] = cpu_baseline(scen, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
