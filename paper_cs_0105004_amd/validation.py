"""Emergent traffic-flow characteristics, measured on the GPU.

The paper validates the driving logic by its macroscopic behaviour (Section
"Macroscopic (emergent) traffic flow characteristics", Figure 4): flow
against density on a 1-lane and a 3-lane freeway, flow through a stop sign
onto a 2-lane road, and flow through a signal that is 30 s red and 30 s
green.  Each sweep here is a batch of independent scenarios stepped
together in one context (one launch per step for all of them):

* ring_diagram: periodic 1-lane rings of L cells, density x slowdown p;
* multilane_diagram: a closed loop of 3-lane links with lane changing;
* stop_sign: a 1-lane side road yielding to a 2-lane main road;
* signal: a 2-lane approach through a fixed-time signal.

Flows are vehicles per step per lane (multiply by 3600 for vehicles per
hour); densities are vehicles per cell.

    python -m paper_cs_0105004_amd.validation      # prints JSON lines
"""
from __future__ import annotations

import json
import sys
from typing import Dict, List, Sequence

import numpy as np

from . import scenarios as S


def _run(scens: Sequence, warm: int, measure: int, tile_lanes: int = 0):
    """Steps every scenario warm + measure steps in one context; returns the
    counters after the warm-up and at the end, per scenario."""
    import torch
    from .sim import Context
    ctx = Context(max_slots=len(scens), tile_lanes=tile_lanes)
    for k, sc in enumerate(scens):
        ctx.load(k, sc)
    slots = list(range(len(scens)))
    ctx.step(slots, warm)
    a = [ctx.stats(k) for k in slots]
    ctx.step(slots, measure)
    b = [ctx.stats(k) for k in slots]
    torch.cuda.synchronize()
    ctx.close()
    return a, b


def ring_diagram(L: int = 1000, densities=None, ps=("0", "0.2", "0.5"),
                 vmax: int = 5, warm: int = 2000, measure: int = 2000,
                 seed: int = 5) -> List[Dict]:
    """Flow (sum of speeds per cell per step) against density on 1-lane
    rings, one ring per (density, p), all in one batch."""
    if densities is None:
        densities = [0.02, 0.05, 0.08, 0.1, 0.12, 0.15, 0.2, 0.3, 0.4, 0.5,
                     0.6, 0.7, 0.8, 0.9]
    scens, keys = [], []
    for p in ps:
        for rho in densities:
            n = max(1, int(round(rho * L)))
            scens.append(S.ring(L, n, vmax, p, seed=seed, T=warm + measure,
                                name=f"ring(rho={rho},p={p})"))
            keys.append((p, n / L))
    a, b = _run(scens, warm, measure)
    out = []
    for (p, rho), sa, sb in zip(keys, a, b):
        flow = (sb["sum_v"] - sa["sum_v"]) / (L * measure)
        out.append({"sweep": "ring", "p": float(p), "density": rho,
                    "flow": flow, "flow_per_hour": flow * 3600})
    return out


def multilane_diagram(lanes: int = 3, link_len: int = 500, n_links: int = 4,
                      densities=None, p: str = "0.2", vmax: int = 5,
                      warm: int = 1500, measure: int = 1500) -> List[Dict]:
    """Flow per lane against density on a closed loop of `lanes`-lane
    links with lane changing (vehicles keep circling)."""
    if densities is None:
        densities = [0.02, 0.05, 0.08, 0.1, 0.15, 0.2, 0.3, 0.5, 0.7]
    cells = link_len * n_links
    scens, keys = [], []
    for rho in densities:
        n = max(1, int(round(rho * cells)))
        scens.append(S.loop_of_links([link_len] * n_links, n, vmax=vmax, p=p,
                                     seed=3, T=warm + measure, lanes=lanes,
                                     placement_seed=11,
                                     flags=S.FLAG_LANE_CHANGE))
        keys.append(n / cells)
    a, b = _run(scens, warm, measure)
    out = []
    for rho, sa, sb in zip(keys, a, b):
        flow = (sb["sum_v"] - sa["sum_v"]) / (cells * lanes * measure)
        lc = (sb["lane_changes"] - sa["lane_changes"]) / measure
        out.append({"sweep": f"loop_{lanes}_lanes", "p": float(p),
                    "density": rho, "flow": flow, "flow_per_hour": flow * 3600,
                    "lane_changes_per_step": lc})
    return out


def _merge_network(main_rate: float, side_rate: float, T: int, seed: int,
                   length: int = 200, p: str = "0.2", signal=None):
    """Main road (2 lanes, rank 0) and a 1-lane side road (rank 1) enter
    node 2 and continue on a 2-lane link.  Vehicles depart as Bernoulli
    streams per step on each approach.  signal = (cycle, red) puts a
    fixed-time plan on the main approach instead and drops the side road's
    demand."""
    rng = np.random.Generator(np.random.PCG64(seed))
    frm = np.array([0, 1, 2], np.int32)
    to = np.array([2, 2, 3], np.int32)
    ln = np.array([length, length, length], np.int32)
    lanes = np.array([2, 1, 2], np.int8)
    rank = np.array([0, 1, 0], np.int8)
    dep_main = np.flatnonzero(rng.random(T) < main_rate)
    dep_side = np.flatnonzero(rng.random(T) < side_rate)
    # two vehicles per step may leave parking on the 2-lane approach
    extra = np.flatnonzero(rng.random(T) < max(0.0, main_rate - 1.0))
    dep_main = np.sort(np.concatenate([dep_main, extra]))
    n_main, n_side = len(dep_main), len(dep_side)
    depart = np.concatenate([dep_main, dep_side]).astype(np.int32)
    n = n_main + n_side
    routes = [[0, 2]] * n_main + [[1, 2]] * n_side
    route_off = np.arange(n + 1, dtype=np.int64) * 2
    xy = np.array([[-1.0, 0.0], [0.0, -1.0], [0.0, 0.0], [1.0, 0.0]])
    sig = {}
    if signal is not None:
        sig = dict(signal_plan=np.array([0, -1, -1], np.int8),
                   plan_cycle=np.array([signal[0]], np.int32),
                   plan_red=np.array([signal[1]], np.int32),
                   plan_offset=np.array([0], np.int32))
    return S.Scenario(
        name="merge", flags=0, vmax=5, slow_thr=S.prob_threshold(p),
        seed=seed, T=T, n_nodes=4, link_from=frm, link_to=to, link_len=ln,
        link_lanes=lanes, link_rank=rank,
        conn_off=np.array([0, 1, 2, 2], np.int64),
        conn_out=np.array([2, 2], np.int32), conn_lo=np.zeros(2, np.int8),
        conn_hi=np.array([1, 0], np.int8), node_xy=xy, n_veh=n,
        depart=depart, route_off=route_off,
        route_links=np.array(routes, np.int32).ravel(), **sig), n_main


def stop_sign(main_rates=None, T: int = 3600, warm: int = 600) -> List[Dict]:
    """Flow of a saturated 1-lane side road through a stop sign (it yields
    to the 2-lane main road) against the main road's flow."""
    if main_rates is None:
        main_rates = [0.0, 0.1, 0.2, 0.3, 0.5, 0.7, 0.9, 1.1, 1.4]
    scens, n_mains = [], []
    for k, r in enumerate(main_rates):
        sc, nm = _merge_network(r, 0.9, T, seed=100 + k)
        scens.append(sc)
        n_mains.append(nm)
    return _merge_flows(scens, n_mains, main_rates, T, warm, "stop_sign")


def signal(demands=None, cycle: int = 60, red: int = 30, T: int = 3600,
           warm: int = 600) -> List[Dict]:
    """Flow through a fixed-time signal (30 s red, 30 s green by default)
    on a 2-lane approach against the demand."""
    if demands is None:
        demands = [0.1, 0.2, 0.4, 0.6, 0.8, 1.0, 1.3, 1.6, 2.0]
    scens, n_mains = [], []
    for k, r in enumerate(demands):
        sc, nm = _merge_network(r, 0.0, T, seed=200 + k, signal=(cycle, red))
        scens.append(sc)
        n_mains.append(nm)
    return _merge_flows(scens, n_mains, demands, T, warm, "signal")


def _merge_flows(scens, n_mains, rates, T, warm, name):
    import torch
    from .sim import Context
    ctx = Context(max_slots=len(scens))
    for k, sc in enumerate(scens):
        ctx.load(k, sc)
    slots = list(range(len(scens)))
    ctx.step(slots, T)
    out = []
    for k, (sc, nm, r) in enumerate(zip(scens, n_mains, rates)):
        ex = ctx.state(k)["exit_t"].reshape(-1, 2)[:, 0]  # leaving approach
        main = ex[:nm]
        side = ex[nm:]
        span = T - warm
        fm = float(((main >= warm) & (main < T)).sum()) / span
        fs = float(((side >= warm) & (side < T)).sum()) / span
        out.append({"sweep": name, "rate": r, "main_flow": fm,
                    "side_flow": fs, "main_per_hour": fm * 3600,
                    "side_per_hour": fs * 3600})
    torch.cuda.synchronize()
    ctx.close()
    return out


def main() -> int:
    import torch
    torch.cuda.set_device(0)
    for fn in (ring_diagram, multilane_diagram, stop_sign, signal):
        for row in fn():
            print(json.dumps(row), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
