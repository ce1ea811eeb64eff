#!/usr/bin/env python3
"""Throughput of the TRANSIMS per-second update on one MI355X.

One step = one simulated second of the whole network (parking insertion,
lane-change sub-step, intersections, car following and move) through the
HIP kernels of libtransims, called via its C ABI.  The default workload is
the Portland-sized synthetic network (77 x 78 grid thinned to 20,024
directed links of 1-3 lanes, 200,000 routed vehicles departing uniformly in
the first 1,800 s, vmax 5, p = 0.2) on its full 3,600-step horizon and full
demand, whatever --steps is.  --steps K is the length of the timed window:
each timed run loads the scenario fresh, advances untimed from t = 0 to the
demand peak t0 (the step with the most vehicles on the network), and times
the K steps [t0, t0 + K) with all inputs resident in HBM; the rate is the
median of 1 + reps runs.  The whole horizon from a fresh load is timed as
well and reported beside it.  As in the paper's series of runs, the same
runs are also timed with the tiling weighted by the link costs an earlier,
untimed run measured (adaptive load balancing).

Prints one JSON line with vehicle-updates/s, the simulated-to-real-time
ratio, the roofline position of the dominant kernel (timed with HIP events
over the window) and the CPU oracle timed on the same window (after
advancing itself from t = 0, untimed), whose counters and state hash at
t0 + K the GPU run must equal.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
METRIC = ("vehicle-updates/sec & sim/real-time ratio (1 GPU, bit-exact); "
          "p50/p99 run latency")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str):
    """The workload at its stated horizon and demand (never shortened)."""
    from paper_cs_0105004_amd import scenarios as S
    if name == "portland":
        scen = S.portland_like()
        cfg = {"workload": "portland_like_grid", "links": scen.n_links,
               "nodes": scen.n_nodes, "lanes": int(scen.link_lanes.sum()),
               "vehicles": scen.n_veh, "horizon_steps": scen.T, "vmax": 5,
               "p": 0.2, "lane_change": False}
    elif name == "portland_signals":
        scen = S.portland_like(signals=(60, 30))
        cfg = {"workload": "portland_like_grid_signals", "links": scen.n_links,
               "nodes": scen.n_nodes, "lanes": int(scen.link_lanes.sum()),
               "vehicles": scen.n_veh, "horizon_steps": scen.T, "vmax": 5,
               "p": 0.2, "lane_change": False,
               "signals": "cycle 60 s, red 30 s, E-W / N-S phases, "
                          "nodes with >= 3 approaches",
               "signalised_links": int((scen.signal_plan >= 0).sum())}
    elif name == "large":
        scen = S.large_network()
        cfg = {"workload": "large_grid_200k_links", "links": scen.n_links,
               "nodes": scen.n_nodes, "lanes": int(scen.link_lanes.sum()),
               "vehicles": scen.n_veh, "horizon_steps": scen.T, "vmax": 5,
               "p": 0.2, "lane_change": True, "turn_lanes": True}
    elif name == "large_quarter":
        # the same generator at a quarter of the grid and the demand: the
        # same kernels and congestion pattern, for counter passes that the
        # full-size network does not complete under the profiler
        scen = S.large_network(scale=0.25)
        cfg = {"workload": "large_grid_quarter_50k_links",
               "links": scen.n_links, "nodes": scen.n_nodes,
               "lanes": int(scen.link_lanes.sum()), "vehicles": scen.n_veh,
               "horizon_steps": scen.T, "vmax": 5, "p": 0.2,
               "lane_change": True, "turn_lanes": True}
    elif name == "ring":
        scen = S.ring()
        cfg = {"workload": "ring_1000_cells", "vehicles": 150,
               "horizon_steps": scen.T, "vmax": 5, "p": 0.2}
    else:
        raise SystemExit(f"unknown workload {name}")
    return scen, cfg


# Algorithmic bytes of the method per step (the lattice formulation: every
# cell of an occupied lane read and written once as int8, each active
# vehicle's int32 id read and written, 16 B per crossing or trip end for its
# route entry, exit time and handoff record, 8 B per vehicle leaving parking):
#   B(t) = 2*C_occ(t) + 8*N(t) + 16*X(t) + 8*I(t)
# The move kernel does the first three terms, the front kernel the last;
# the one-kernel step does all four.
def algorithmic_bytes(kind, st):
    if kind == "back":
        return (2.0 * st["c_occ"] + 8.0 * st["veh_updates"]
                + 16.0 * (st["crossings"] + st["exits"]))
    if kind == "front":
        return 8.0 * st["insertions"]
    if kind == "step":  # one kernel does the whole step
        return (2.0 * st["c_occ"] + 8.0 * st["veh_updates"]
                + 16.0 * (st["crossings"] + st["exits"])
                + 8.0 * st["insertions"])
    return 2.0 * st["c_occ"] + 8.0 * st["veh_updates"]  # ring: one launch


# the sources each kernel family compiles from: a family's digest changes
# only when its own code (or a shared header) does
_SHARED = ("device.h", "kernels.h", "layout.h", "philox.h")
KERNEL_SOURCES = {"step": ("step.hip",) + _SHARED,
                  "front_back": ("front_back.hip",) + _SHARED,
                  "ring": ("ring_stats.hip",) + _SHARED}
FAMILY = {"step": "step", "front": "front_back", "back": "front_back",
          "ring": "ring"}


def _code_only(text: str) -> str:
    """The source without comments, trailing blanks and empty lines, so that
    a comment edit does not change what counts as the measured code."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.split("\n"))
    return "\n".join(ln for ln in lines if ln)


def kernel_digest(family: str = "step") -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, "paper_cs_0105004_amd", "csrc", f),
                  encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def family_of(kinds) -> str:
    """Kernel family of the step kernels that ran ("front"/"back" together
    are the two-kernel family)."""
    fams = {FAMILY[k] for k in kinds}
    return fams.pop() if len(fams) == 1 else "front_back"


# HBM bytes per launch of the step kernel, by workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over the dispatches of
# the timed window) scaled by what the same counters read for a plain copy
# of known size (x 2.0 and x 1.0).  Valid only for the kernel sources with
# this digest (of the kernel's family) and for exactly that window and tile
# shape; any other run reports null.
MEASURED_TRAFFIC = {
    "800401fd3b3c1d68": {  # step.hip family
        "portland": [
            # k_step<false, false>, the default 16-lane / 1,024-cell tiles,
            # window [1800, 1820): FETCH 3277.6 KiB x 2.0 + WRITE 2272.0 KiB
            {"window": (1800, 20), "tiles": (16, 1024),
             "bytes_per_launch": 8827.2 * 1024},
            # window [1800, 1900): FETCH 3154.7 x 2.0 + WRITE 2175.0
            {"window": (1800, 100), "tiles": (16, 1024),
             "bytes_per_launch": 8484.4 * 1024},
        ],
        "batched": [
            # k_step<true, false>, 64 replications, 64-lane / 12,288-cell
            # tiles, window [1800, 1900): FETCH 52428.6 KiB x 2.0 + WRITE
            # 34034.8 KiB x 1.0
            {"window": (1800, 100), "tiles": (64, 12288),
             "bytes_per_launch": 138892.0 * 1024},
        ],
    },
    "00c4255505f63b72": {  # front_back.hip family (lane change + move)
        "large_quarter": [
            # per step, default 32-lane / 4,096-cell tiles, window
            # [7100, 7200): k_front FETCH 7863.3 KiB x 2.0 + WRITE 2498.5
            # KiB; k_back FETCH 6798.5 x 2.0 + WRITE 5631.5
            {"window": (7100, 100), "tiles": (32, 4096),
             "bytes_per_launch": 37453.6 * 1024},
        ],
    },
}


def measured_traffic(family: str, workload: str, window, tiles=(0, 0)):
    """The measured bytes per launch for this kernel family, workload,
    timed window (t0, K) and (tile_lanes, tile_cells) (0: the library
    default), if the counters were taken on exactly that."""
    for tr in MEASURED_TRAFFIC.get(kernel_digest(family), {}).get(workload, ()):
        if (tuple(tr["window"]) == tuple(window)
                and tuple(tr["tiles"]) == tuple(tiles)):
            return tr["bytes_per_launch"]
    return None


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
    budget_s seconds of CPU time have been spent (used where the oracle
    cannot reach the timed window within the budget)."""
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
                      f"single thread; the timed window lies beyond what the "
                      f"oracle reaches in the budget)",
            "host": host_info()}, st


def cpu_window(scen, t0: int, k: int, budget_s: float, max_reps: int = 20):
    """The oracle on the timed window: it advances itself from t = 0 to t0
    (untimed) and is timed over the K steps [t0, t0 + K); further passes
    over the same window restart from its own saved state at t0 (a restart
    equals the uninterrupted run) until about budget_s seconds of stepping
    have been timed.  Returns the baseline object and the oracle's counters
    at t0 + K of the first pass."""
    import oracle
    o = oracle.OracleSim(scen)
    a0 = time.perf_counter()
    o.step(t0)
    adv = time.perf_counter() - a0
    saved = scen.with_state(o.state(), t0)
    st0 = o.stats()
    t1 = time.perf_counter()
    o.step(k)
    timed = time.perf_counter() - t1
    end = o.stats()
    o.close()
    upd = end["veh_updates"] - st0["veh_updates"]
    total_upd, passes = upd, 1
    while timed < budget_s and passes < max_reps:
        r = oracle.OracleSim(saved)
        t1 = time.perf_counter()
        r.step(k)
        timed += time.perf_counter() - t1
        again = r.stats()
        r.close()
        assert again["hash"] == end["hash"], "oracle restart diverged"
        total_upd += upd
        passes += 1
    return {"value": total_upd / timed, "unit": "vehicle-updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"the timed window, steps {t0}..{t0 + k - 1} of the "
                      f"same workload, {passes} pass(es) ({total_upd} "
                      f"vehicle-updates, {timed:.2f} s stepping, single "
                      f"thread), after advancing untimed from t = 0 "
                      f"({adv:.1f} s)",
            "host": host_info()}, end


def oracle_check(ctx, scen, ost, link_cost=None) -> dict:
    """The GPU from a fresh load to the step the oracle reached: every
    counter and the state hash must be equal."""
    ctx.load(0, scen, link_cost=link_cost)
    ctx.step(0, int(ost["t"]))
    gst = ctx.stats(0)
    diff = sorted(k for k in ost if gst.get(k) != ost[k])
    return {"steps": int(ost["t"]), "state_hash": f"{ost['hash']:016x}",
            "equal": not diff, "differing": diff}


def roofline_from(kt, stats_list, region_ms=None, workload=None, window=None,
                  tiles=(0, 0)):
    """Roofline object of the dominant step kernel from per-kernel times and
    the summed counters of the scenarios it processed.  With one step kernel
    and the event time of the timed region, the launch duration is that
    time per launch; otherwise the event-node times of a profiled replay."""
    kinds = [k for k in ("front", "back", "ring", "step") if kt[k][0] > 0]
    if not kinds:
        return None
    tot = {k: sum(st[k] for st in stats_list)
           for k in ("c_occ", "veh_updates", "crossings", "exits",
                     "insertions")}
    dom = max(kinds, key=lambda k: kt[k][1])
    launches = kt[dom][0]
    name = f"k_{dom}"
    if region_ms is not None:
        avg_ms = region_ms / launches
        timing = "events around the timed window / launches"
        if len(kinds) > 1:
            dom, name = "step", "k_front + k_back"
            timing += " (lane-change and move kernels together)"
    else:
        avg_ms = kt[dom][1] / launches
        timing = "event nodes between kernels (corrected)"
    bytes_launch = algorithmic_bytes(dom, tot) / launches
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    fam = family_of(kinds)
    traffic = (measured_traffic(fam, workload, window, tiles)
               if workload and window else None)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_note": (
                "rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB per "
                "dispatch over this window (copy-calibrated)"
                if traffic is not None else
                "null: no counter pass of these kernel sources on this "
                "window and tile shape"),
            "kernel": name, "avg_launch_us": avg_ms * 1e3,
            "timing": timing,
            "algorithmic_bytes_per_launch": bytes_launch,
            "kernel_sources_digest": kernel_digest(fam),
            "kernel_ms": {k: kt[k][1] for k in kinds},
            "launches": {k: kt[k][0] for k in kinds}}


def host_info() -> dict:
    """CPU model and core counts of the host the oracle runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "usable_cores": usable}


def oracle_all_cores(scens, budget_s: float, max_workers: int = 16):
    """The host's aggregate oracle rate over independent scenarios: one
    thread per scenario (the oracle is C called through ctypes, which
    releases the GIL while it steps), each from its start, for about
    budget_s seconds.  At most max_workers threads (the host's share for
    one GPU)."""
    import threading
    import oracle
    n = max(1, min(max_workers, host_info()["usable_cores"] or 1, len(scens)))
    sims = [oracle.OracleSim(sc) for sc in scens[:n]]  # created one by one
    done = [0] * n
    t0 = time.perf_counter()
    stop = t0 + budget_s

    def run(k):
        sc = scens[k]
        while time.perf_counter() < stop and done[k] < sc.T:
            m = min(25, sc.T - done[k])
            sims[k].step(m)
            done[k] += m

    threads = [threading.Thread(target=run, args=(k,)) for k in range(n)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    dt = time.perf_counter() - t0
    upd = sum(o.stats()["veh_updates"] for o in sims)
    for o in sims:
        o.close()
    return {"value": upd / dt, "unit": "vehicle-updates/s", "cores": n,
            "kind": "oracle",
            "sample": f"{n} scenario(s) of the same workload, one thread "
                      f"each, from t = 0, {sum(done)} scenario-steps "
                      f"({upd} vehicle-updates, {dt:.1f} s)",
            "vehicle_updates": upd, "host": host_info()}


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """GB/s of a plain device-to-device copy of nbytes (bytes read plus
    bytes written), the best of reps: the reachable HBM rate, beside the
    published peak."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def with_copy_reference(roof):
    """Adds the measured copy bandwidth and the fraction of it achieved."""
    if roof is not None:
        cg = copy_bandwidth()
        roof["copy_gbs"] = cg
        roof["frac_of_copy"] = roof["achieved"] / cg
    return roof


def oracle_sample(scens, budget_s: float):
    """The oracle over the given scenarios one after another (each from its
    start) until about budget_s seconds of CPU time are spent."""
    import oracle
    t0 = time.perf_counter()
    upd, steps, used = 0, 0, 0
    finals = []
    for sc in scens:
        o = oracle.OracleSim(sc)
        done = 0
        while time.perf_counter() - t0 < budget_s and done < sc.T:
            k = min(25, sc.T - done)
            o.step(k)
            done += k
        finals.append(o.stats())
        upd += finals[-1]["veh_updates"]
        steps += done
        used += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": upd / dt, "unit": "vehicle-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{used} scenario(s) of the same workload from t = 0, "
                      f"{steps} scenario-steps ({upd} vehicle-updates, "
                      f"{dt:.1f} s, single thread)",
            "host": host_info()}, finals


def bench_batched(args):
    """64 independent replications of uneven size in one context, stepped
    together (one launch per sub-step for all of them, HIP graphs,
    autotuned tiling), against the plain loop: the same kernels run one
    scenario at a time, one launch per sub-step, no graph.  The scenarios
    keep their 3,600-step horizon and demand; the timed window is --steps
    steps at the step where the most vehicles are on the networks."""
    import torch
    from paper_cs_0105004_amd import scenarios as S
    from paper_cs_0105004_amd.autotune import autotune
    from paper_cs_0105004_amd.sim import Context
    log("bench: generating 64 replications")
    scens = S.batched_scenarios()
    n = len(scens)
    T, K = scens[0].T, args.steps
    if not 1 <= K <= T:
        raise SystemExit(f"--steps must be 1..{T}")
    slots = list(range(n))
    if args.tile_lanes and args.tile_cells:
        # a fixed configuration (e.g. for counter runs, where the profiler
        # distorts the tuner's timings)
        tune = {"tile_lanes": args.tile_lanes, "tile_cells": args.tile_cells,
                "back_pieces": 1, "graph_steps": args.graph_steps or 64,
                "trials": "skipped (fixed configuration)"}
    else:
        log("bench: autotuning")
        # trials at the demand peak (mid-horizon), where the step costs most
        tune = autotune(scens, warm_steps=T // 2, trial_steps=128, reps=2,
                        log=log)
    ctx = Context(max_slots=n, tile_lanes=tune["tile_lanes"],
                  back_pieces=tune["back_pieces"],
                  graph_steps=tune["graph_steps"],
                  tile_cells=tune["tile_cells"], step_mode=args.step_mode)

    def load_all(cs):
        for k, sc in enumerate(scens):
            ctx.load(k, sc, link_cost=cs[k])
        torch.cuda.synchronize()

    load_all([None] * n)
    ctx.step(slots, args.warmup)
    torch.cuda.synchronize()
    # the demand peak of the batch
    log("bench: locating the demand peak")
    load_all([None] * n)
    t_peak, n_peak, t = 0, -1, 0
    while t < T:
        m = min(50, T - t)
        ctx.step(slots, m)
        t += m
        a = sum(ctx.stats(k)["n_active"] for k in slots)
        if a > n_peak:
            t_peak, n_peak = t, a
    t0 = min(max(t_peak, K), T - K)
    # adaptive load balancing: an untimed run of the whole horizon measures
    # every slot's link costs; a second set of timed runs is tiled with them
    costs = [None] * n
    if not args.no_feedback:
        log(f"bench: cost-measuring run of {T} batched steps")
        load_all([None] * n)
        ctx.step(slots, T)
        costs = [ctx.link_costs(k) for k in slots]

    def window_run(cs):
        load_all(cs)
        if t0 > K:
            ctx.step(slots, t0 - K)
        ctx.step(slots, K)  # builds the graph the window replays
        st_a = [ctx.stats(k) for k in slots]
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t1 = time.perf_counter()
        ev0.record(ctx.stream)
        ctx.step(slots, K)
        ev1.record(ctx.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        return wall, ev0.elapsed_time(ev1), st_a, [ctx.stats(k) for k in slots]

    def window_runs(cs):
        runs = [window_run(cs) for _ in range(1 + max(args.reps, 0))]
        assert len({tuple(s["hash"] for s in r[3]) for r in runs}) == 1, \
            "repeat diverged"
        return sorted(runs, key=lambda r: r[0])[len(runs) // 2], runs

    def full_runs(cs):
        walls, st = [], None
        for _ in range(1 + max(args.reps, 0)):
            load_all(cs)
            t1 = time.perf_counter()
            ctx.step(slots, T)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t1)
            st1 = [ctx.stats(k) for k in slots]
            assert st is None or [a["hash"] for a in st] == \
                [b["hash"] for b in st1], "diverged"
            st = st1
        return sorted(walls), st

    def pct(walls, q):
        return walls[min(len(walls) - 1, int(round(q * (len(walls) - 1))))]

    def delta(a, b, key):
        return sum(y[key] - x[key] for x, y in zip(a, b))

    log(f"bench: timing the window [{t0}, {t0 + K}) of all {n} scenarios, "
        f"{1 + max(args.reps, 0)} runs")
    (wall, region_ms, st_a, st_b), runs = window_runs([None] * n)
    win_upd = delta(st_a, st_b, "veh_updates")
    win = [{k: y[k] - x[k] for k in ("veh_updates", "sum_v", "crossings",
                                     "exits", "insertions", "c_occ")}
           for x, y in zip(st_a, st_b)]
    log(f"bench: timing the whole horizon, {1 + max(args.reps, 0)} runs")
    fwalls, fst = full_runs([None] * n)
    fupd = sum(s["veh_updates"] for s in fst)
    full = {"value": fupd / pct(fwalls, 0.5),
            "ms_per_step": pct(fwalls, 0.5) * 1e3 / T,
            "sim_real_time_ratio_per_scenario": T / pct(fwalls, 0.5),
            "vehicle_updates": fupd,
            "run_latency_ms": {"p50": pct(fwalls, 0.5) * 1e3,
                               "p99": pct(fwalls, 0.99) * 1e3,
                               "runs": len(fwalls)}}
    fed = None
    if not args.no_feedback:
        log("bench: the same runs with cost feedback")
        (cwall, _, _, cst), _ = window_runs(costs)
        assert [a["hash"] for a in cst] == [b["hash"] for b in st_b]
        cfw, cfst = full_runs(costs)
        assert [a["hash"] for a in cfst] == [b["hash"] for b in fst]
        fed = {"value": win_upd / cwall, "ms_per_step": cwall * 1e3 / K,
               "full_horizon": {"value": fupd / pct(cfw, 0.5),
                                "ms_per_step": pct(cfw, 0.5) * 1e3 / T}}
    log("bench: plain loop")
    plain = Context(max_slots=1, graph_steps=-1)
    pwall, pupd, pfwall = 0.0, 0, 0.0
    for k, sc in enumerate(scens):
        plain.load(0, sc)
        plain.step(0, t0)
        plain.stats(0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain.step(0, K)
        torch.cuda.synchronize()
        pwall += time.perf_counter() - t1
        st = plain.stats(0)
        assert st["hash"] == st_b[k]["hash"], "plain loop diverged"
        pupd += st["veh_updates"] - st_a[k]["veh_updates"]
        plain.load(0, sc)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain.step(0, T)
        torch.cuda.synchronize()
        pfwall += time.perf_counter() - t1
        assert plain.stats(0)["hash"] == fst[k]["hash"], "plain loop diverged"
    plain.close()
    # kernel times of the same window, replayed with events (the last step
    # kernels this process runs)
    load_all([None] * n)
    ctx.step(slots, t0)
    for k in slots:
        ctx.stats(k)
    ctx.profile(True)
    ctx.step(slots, K)
    kt = ctx.kernel_times()
    ctx.profile(False)
    for k in slots:
        assert ctx.stats(k)["hash"] == st_b[k]["hash"], "replay diverged"
    roof = roofline_from(kt, win, region_ms, workload="batched",
                         window=(t0, K),
                         tiles=(tune["tile_lanes"], tune["tile_cells"]))
    roof = with_copy_reference(roof)
    ctx.close()
    cfg = {"workload": "batched_64_replications", "scenarios": n,
           "links": int(sum(sc.n_links for sc in scens)),
           "lanes": int(sum(int(sc.link_lanes.sum()) for sc in scens)),
           "vehicles": int(sum(sc.n_veh for sc in scens)),
           "horizon_steps": T, "vmax": 5, "p": 0.2,
           "tile_lanes": tune["tile_lanes"], "tile_cells": tune["tile_cells"],
           "graph_steps": tune["graph_steps"], "timed_window": [t0, t0 + K],
           "peak_active": n_peak, "peak_step": t_peak}
    walls = sorted(r[0] for r in runs)
    out = {"metric": METRIC, "value": win_upd / wall,
           "unit": "vehicle-updates/s",
           "n_gpus": 1, "steps": K, "warmup": args.warmup,
           "ms_per_step": wall * 1e3 / K,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int32", "data": "synthetic", "config": cfg,
           "timed_window": [t0, t0 + K],
           "sim_real_time_ratio_per_scenario": K / wall,
           "vehicle_updates": win_upd, "wall_s": wall, "event_ms": region_ms,
           "run_latency_ms": {"p50": pct(walls, 0.5) * 1e3,
                              "p99": pct(walls, 0.99) * 1e3,
                              "runs": len(walls),
                              "what": "the timed window of each run"},
           "full_horizon": full,
           "load_balancing": "tiles ordered by the load the routes plan",
           "with_feedback": fed,
           "plain_loop": {"value": pupd / pwall, "wall_s": pwall,
                          "full_horizon_value": fupd / pfwall,
                          "full_horizon_wall_s": pfwall},
           "speedup_vs_plain_loop": (win_upd / wall) / (pupd / pwall),
           "speedup_vs_plain_loop_full_horizon":
               (fupd / pct(fwalls, 0.5)) / (fupd / pfwall),
           "autotune": tune["trials"], "roofline": roof}
    if not args.no_cpu_baseline:
        log(f"bench: oracle on the window of the first scenarios "
            f"({args.cpu_seconds:.0f} s budget)")
        t1 = time.perf_counter()
        upd, dt, checks = 0, 0.0, []
        for k, sc in enumerate(scens):
            base, ost = cpu_window(sc, t0, K, 0.0, max_reps=1)
            u = ost["veh_updates"] - st_a[k]["veh_updates"]
            upd += u
            dt += u / base["value"]
            checks.append({"scenario": k, "steps": int(ost["t"]),
                           "equal": all(st_b[k].get(c) == ost[c]
                                        for c in ost)})
            if time.perf_counter() - t1 >= args.cpu_seconds:
                break
        out["cpu_baseline"] = {
            "value": upd / dt, "unit": "vehicle-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"the timed window, steps {t0}..{t0 + K - 1}, of the "
                      f"first {len(checks)} scenario(s), one after another "
                      f"({upd} vehicle-updates, {dt:.2f} s stepping, single "
                      f"thread), each after advancing untimed from t = 0",
            "host": host_info()}
        out["oracle_check"] = {"equal": all(c["equal"] for c in checks),
                               "scenarios": checks,
                               "what": "every counter and the state hash at "
                                       "the end of the window"}
        log(f"bench: oracle on all host cores ({args.cpu_seconds:.0f} s)")
        out["cpu_all_cores"] = oracle_all_cores(scens, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(args):
    """Poisson arrivals (4 per second over 60 s) of runs drawn from 32
    pre-generated (network, demand) sets of 1k-50k links, served by the
    continuous-batching loop; p50/p99 completion latency and aggregate
    vehicle-updates/s.  A second, shorter pass with kernel timing gives the
    roofline position."""
    import torch
    from paper_cs_0105004_amd import scenarios as S
    from paper_cs_0105004_amd.serve import Server, poisson_trace, summarize
    from paper_cs_0105004_amd.sim import Context
    log("bench: generating the request pool")
    pool = S.serving_pool()
    trace = poisson_trace(pool, rate_per_s=4.0, window_s=args.window)
    # warm-up: a few requests through a throw-away server
    srv = Server(max_slots=64, chunk=64)
    srv.run(trace[:4], realtime=False)
    torch.cuda.synchronize()
    log(f"bench: serving {len(trace)} requests")
    t0 = time.perf_counter()
    res = srv.run(trace, realtime=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    srv.close()
    summ = summarize(res, wall)
    # a few results checked against the same run alone
    check = Context(max_slots=1)
    for r in res[:: max(1, len(res) // 4)]:
        sc = trace[r.rid].scen
        check.load(0, sc)
        check.step(0, sc.T)
        assert check.stats(0)["hash"] == r.stats["hash"], "mix != alone"
    check.close()
    # kernel timing over the first 15 s of the same trace
    short = [q for q in trace if q.arrival_s <= 15.0]
    srv = Server(max_slots=64, chunk=64)
    srv.ctx.profile(True)
    res2 = srv.run(short, realtime=True)
    kt = srv.ctx.kernel_times()
    srv.close()
    roof = with_copy_reference(roofline_from(kt, [r.stats for r in res2]))
    cfg = {"workload": "serving_poisson", "rate_per_s": 4.0,
           "window_s": args.window, "requests": len(trace), "pool_sets": 32,
           "links_range": [1000, 50000], "vehicles_per_link": 10,
           "horizon_range": [600, 3600], "max_slots": 64, "chunk_steps": 64}
    out = {"metric": METRIC, "value": summ["updates_per_s"],
           "unit": "vehicle-updates/s", "n_gpus": 1, "steps": None,
           "warmup": 4, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic", "config": cfg,
           "p50_latency_s": summ["p50_latency_s"],
           "p99_latency_s": summ["p99_latency_s"],
           "max_latency_s": summ["max_latency_s"],
           "vehicle_updates": summ["vehicle_updates"], "wall_s": wall,
           "roofline": roof}
    if not args.no_cpu_baseline:
        log(f"bench: oracle sample ({args.cpu_seconds:.0f} s budget)")
        out["cpu_baseline"], _ = oracle_sample([q.scen for q in trace[:3]],
                                               args.cpu_seconds)
        log(f"bench: oracle on all host cores ({args.cpu_seconds:.0f} s)")
        out["cpu_all_cores"] = oracle_all_cores([q.scen for q in trace[:16]],
                                                args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="length of the timed window at the demand peak "
                         "(batched: of the window of all scenarios)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="portland")
    ap.add_argument("--tile-lanes", type=int, default=0)
    ap.add_argument("--tile-cells", type=int, default=0)
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="batched: steps per graph with --tile-lanes and "
                         "--tile-cells (which skip the autotuner)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-feedback", action="store_true",
                    help="skip the cost-measuring run and the runs tiled "
                         "with its costs")
    ap.add_argument("--reps", type=int, default=5,
                    help="further runs of K steps (the rate is the median "
                         "run's; the runs give the latency percentiles)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    metavar="BYTES", help="only run plain copies of BYTES")
    ap.add_argument("--window", type=float, default=60.0,
                    help="serving: seconds of Poisson arrivals")
    ap.add_argument("--step-mode", type=int, default=0,
                    help="the library's step_mode (2: the one-kernel step "
                         "skips idle lanes); single and batched workloads")
    ap.add_argument("--counter-pass", action="store_true",
                    help="only the timed window once (fresh load, untimed "
                         "advance to the demand peak, K steps), for a "
                         "rocprofv3 counter run: the window's launches are "
                         "the last K of the step kernels")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not "
              f"supported (scenarios are independent and would shard by "
              f"slot across GPUs; this build runs on one)", file=sys.stderr)
        return 2

    import torch

    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        return copy_calibration(args.copy_calibration)
    if args.counter_pass:
        return counter_pass(args)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "serve":
        return bench_serve(args)
    return bench_single(args)


def counter_pass(args):
    """The timed window of the workload once and nothing after it, so that
    a profiler's last K dispatches of the step kernels are exactly the
    window's (no timing, no oracle)."""
    from paper_cs_0105004_amd import scenarios as S
    from paper_cs_0105004_amd.sim import Context
    K = args.steps
    if args.workload == "batched":
        scens = S.batched_scenarios()
        tiles = dict(tile_lanes=args.tile_lanes or 64,
                     tile_cells=args.tile_cells or 8192,
                     graph_steps=args.graph_steps or 64)
    else:
        scens = [make_workload(args.workload)[0]]
        tiles = dict(tile_lanes=args.tile_lanes, tile_cells=args.tile_cells)
    n = len(scens)
    slots = list(range(n))
    ctx = Context(max_slots=n, step_mode=args.step_mode, **tiles)
    for k, sc in enumerate(scens):
        ctx.load(k, sc)
    T = scens[0].T
    best, t_peak, t = -1, 0, 0
    log("counter pass: locating the demand peak")
    while t < T:
        m = min(50, T - t)
        ctx.step(slots, m)
        t += m
        a = sum(ctx.stats(k)["n_active"] for k in slots)
        if a > best:
            best, t_peak = a, t
        if t % 1000 == 0:
            log(f"counter pass: t = {t}")
    t0 = min(max(t_peak, K), T - K)
    for k, sc in enumerate(scens):
        ctx.load(k, sc)
    log(f"counter pass: advancing to t = {t0}")
    done = 0
    while done < t0:
        m = min(1000, t0 - done)
        ctx.step(slots, m)
        done += m
        ctx.stats(0)
        log(f"counter pass: t = {done}")
    st_a = [ctx.stats(k) for k in slots]
    log(f"counter pass: the window [{t0}, {t0 + K})")
    ctx.step(slots, K)
    st_b = [ctx.stats(k) for k in slots]
    win = {c: sum(b[c] - a[c] for a, b in zip(st_a, st_b))
           for c in ("veh_updates", "c_occ", "crossings", "exits",
                     "insertions")}
    print(json.dumps({"counter_pass": args.workload, "window": [t0, t0 + K],
                      "tiles": tiles, "window_counters": win,
                      "algorithmic_bytes_per_step":
                          algorithmic_bytes("step", win) / K}), flush=True)
    ctx.close()
    return 0


def find_peak(ctx, scen, every: int = 50):
    """The step, a multiple of `every`, at which the most vehicles are on
    the network, from one untimed run of the horizon (every result equals
    the oracle's, so this choice does not depend on the device)."""
    ctx.load(0, scen)
    best_n, best_t, t = -1, 0, 0
    while t < scen.T:
        k = min(every, scen.T - t)
        ctx.step(0, k)
        t += k
        n = ctx.stats(0)["n_active"]
        if n > best_n:
            best_n, best_t = n, t
    return best_t, best_n


def bench_single(args):
    """One scenario: the timed window of --steps steps at the demand peak,
    and the whole horizon, each from a fresh load."""
    import torch
    from paper_cs_0105004_amd.sim import Context
    log(f"bench: generating workload {args.workload}")
    scen, cfg = make_workload(args.workload)
    T, K = scen.T, args.steps
    if not 1 <= K <= T:
        raise SystemExit(f"--steps must be 1..{T} (the window inside the "
                         f"horizon)")
    ctx = Context(max_slots=2, tile_lanes=args.tile_lanes,
                  tile_cells=args.tile_cells, step_mode=args.step_mode)

    # warm-up on a throw-away copy
    log(f"bench: warmup {args.warmup} steps")
    ctx.load(1, scen)
    ctx.step(1, args.warmup)
    ctx.stats(1)
    ctx.unload(1)
    log("bench: locating the demand peak")
    t_peak, n_peak = find_peak(ctx, scen)
    t0 = min(max(t_peak, K), T - K)
    # adaptive load balancing, the paper's feedback between runs: an untimed
    # run of the whole horizon measures every link's cost, and a second set
    # of timed runs is tiled with those costs (--no-feedback: skip it)
    costs = None
    if not args.no_feedback and args.workload != "ring":
        log(f"bench: cost-measuring run of {T} steps")
        ctx.load(1, scen)
        ctx.step(1, T)
        ctx.stats(1)
        costs = ctx.link_costs(1)
        ctx.unload(1)

    def ev_pair():
        return (torch.cuda.Event(enable_timing=True),
                torch.cuda.Event(enable_timing=True))

    def window_run(link_cost):
        """Fresh load, untimed advance to t0 (its last K steps build the
        graph the window replays), then the K timed steps: wall time, the
        time between HIP events on the library's stream, and the counters
        at t0 and at t0 + K."""
        ctx.load(0, scen, link_cost=link_cost)
        if t0 > K:
            ctx.step(0, t0 - K)
        ctx.step(0, K)
        st_a = ctx.stats(0)
        torch.cuda.synchronize()
        ev0, ev1 = ev_pair()
        t1 = time.perf_counter()
        ev0.record(ctx.stream)
        ctx.step(0, K)
        ev1.record(ctx.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        return wall, ev0.elapsed_time(ev1), st_a, ctx.stats(0)

    def window_runs(link_cost):
        runs = [window_run(link_cost) for _ in range(1 + max(args.reps, 0))]
        assert len({r[3]["hash"] for r in runs}) == 1, "repeat diverged"
        return sorted(runs, key=lambda r: r[0])[len(runs) // 2], runs

    def full_run(link_cost):
        ctx.load(0, scen, link_cost=link_cost)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.step(0, T)
        torch.cuda.synchronize()
        return time.perf_counter() - t1, ctx.stats(0)

    def full_runs(link_cost):
        runs = [full_run(link_cost) for _ in range(1 + max(args.reps, 0))]
        assert len({r[1]["hash"] for r in runs}) == 1, "repeat diverged"
        walls = sorted(r[0] for r in runs)
        return walls, runs[0][1]

    def pct(walls, q):
        return walls[min(len(walls) - 1, int(round(q * (len(walls) - 1))))]

    log(f"bench: timing the window [{t0}, {t0 + K}), "
        f"{1 + max(args.reps, 0)} runs")
    (wall, region_ms, st_a, st_b), runs = window_runs(None)
    win = {k: st_b[k] - st_a[k] for k in ("veh_updates", "sum_v", "crossings",
                                          "exits", "insertions", "c_occ",
                                          "lane_changes")}
    value = win["veh_updates"] / wall
    log(f"bench: timing the whole horizon, {1 + max(args.reps, 0)} runs")
    fwalls, fst = full_runs(None)
    fmed = pct(fwalls, 0.5)
    full = {"value": fst["veh_updates"] / fmed,
            "ms_per_step": fmed * 1e3 / T, "sim_real_time_ratio": T / fmed,
            "vehicle_updates": fst["veh_updates"],
            "run_latency_ms": {"p50": fmed * 1e3,
                               "p99": pct(fwalls, 0.99) * 1e3,
                               "runs": len(fwalls)},
            "bit_exact_state_hash": f"{fst['hash']:016x}"}
    fed = None
    if costs is not None:
        log("bench: the same runs with cost feedback")
        (cwall, _, _, cst), _ = window_runs(costs)
        assert cst["hash"] == st_b["hash"], "feedback changed the result"
        cfw, cfst = full_runs(costs)
        assert cfst["hash"] == fst["hash"], "feedback changed the result"
        fed = {"value": win["veh_updates"] / cwall,
               "ms_per_step": cwall * 1e3 / K,
               "full_horizon": {"value": cfst["veh_updates"] / pct(cfw, 0.5),
                                "ms_per_step": pct(cfw, 0.5) * 1e3 / T}}

    # kernel timing pass over the same window: its K steps inside a HIP
    # graph with an event between every two kernels on the library's stream
    # (the last step kernels this process runs, so a rocprofv3 kernel trace
    # of this command ends with exactly these K launches)
    ctx.load(0, scen)
    if t0 > 0:
        ctx.step(0, t0)
    ctx.stats(0)
    ctx.profile(True)
    ctx.step(0, K)
    kt = ctx.kernel_times()
    ctx.profile(False)
    assert ctx.stats(0)["hash"] == st_b["hash"], "timing pass diverged"
    tiling = ctx.tiling(0)
    # the tile shape the traffic was measured with: the library's defaults
    # (16 lanes / 1,024 cells for one-kernel scenarios, 32 / 4,096 with lane
    # changes) unless given
    lc = args.workload in ("large", "large_quarter")
    tiles = (args.tile_lanes or (32 if lc else 16),
             args.tile_cells or (4096 if lc else 1024))
    roof = roofline_from(kt, [win], region_ms, workload=args.workload,
                         window=(t0, K), tiles=tiles)
    with_copy_reference(roof)
    walls = sorted(r[0] for r in runs)
    cfg = dict(cfg, timed_window=[t0, t0 + K], peak_active=n_peak,
               peak_step=t_peak)
    out = {
        "metric": METRIC, "value": value, "unit": "vehicle-updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic", "config": cfg,
        "timed_window": [t0, t0 + K],
        "sim_real_time_ratio": K / wall,
        "vehicle_updates": win["veh_updates"], "wall_s": wall,
        "event_ms": region_ms,
        "bit_exact_state_hash": f"{st_b['hash']:016x}",
        "run_latency_ms": {"p50": pct(walls, 0.5) * 1e3,
                           "p99": pct(walls, 0.99) * 1e3, "runs": len(walls),
                           "what": "the timed window of each run"},
        "full_horizon": full,
        "load_balancing": "tiles ordered by the load the routes plan",
        "with_feedback": fed,
        "tiling": {"tiles": tiling["n_tiles"], "e_dmn": tiling["e_dmn"],
                   "e_tile": tiling["e_tile"]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        if args.workload in ("large", "large_quarter"):
            # the oracle would need most of an hour to reach the peak of the
            # 200,000-link network (a quarter of that for the quarter-size
            # one): it is timed on its first steps instead, and the GPU is
            # checked against it where it stopped
            log(f"bench: oracle sample ({args.cpu_seconds:.0f} s budget)")
            out["cpu_baseline"], ost = cpu_baseline(scen, args.cpu_seconds)
            log(f"bench: GPU against the oracle at step {ost['t']}")
            out["oracle_check"] = oracle_check(ctx, scen, ost)
        else:
            log(f"bench: oracle on the window (advance to {t0}, then "
                f"{args.cpu_seconds:.0f} s budget)")
            out["cpu_baseline"], ost = cpu_window(scen, t0, K,
                                                  args.cpu_seconds)
            # the GPU's counters at t0 + K of the timed runs (fresh load,
            # all counters from t = 0) against the oracle's
            diff = sorted(k for k in ost if st_b.get(k) != ost[k])
            out["oracle_check"] = {"steps": int(ost["t"]),
                                   "state_hash": f"{ost['hash']:016x}",
                                   "equal": not diff, "differing": diff,
                                   "what": "every counter and the state "
                                           "hash at the end of the window"}
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
