"""Iteration series: runs of the micro-simulation fed back through routing.

The paper's production use is a relaxation: the micro-simulation runs about
fifty times, and between runs a fraction of the travellers get new routes
computed from the link travel times the last run produced (Section
"Introduction"; Section "Other modules").  The same series is also where
the paper applies adaptive load balancing: the execution times measured in
one run weight the domain decomposition of the next (Section "Adaptive
Load Balancing").  This module runs that loop with the GPU library doing
every micro-simulation and the host doing the re-routing:

* run r simulates the current plans for the horizon;
* each link's travel time is the mean time its travellers spent on it
  (from the exit times; the link's free-flow time if nobody used it);
* a seeded random `reroute` fraction of the travellers get the shortest
  path between their origin and destination under those times;
* the next run is tiled with the per-link costs the GPU measured in run r.

Every run is a normal scenario, so its result equals the CPU oracle's for
the same plans.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import scenarios as S


def link_travel_times(scen, exit_t: np.ndarray) -> np.ndarray:
    """Mean steps spent on each link in a run: a traveller that left route
    entry j-1 in step a and entry j in step b spent b - a steps on link j.
    Entries a run did not finish, and first links (whose entry time
    includes the wait in parking), do not count; a link nobody finished
    gets its free-flow time len / vmax."""
    L = scen.n_links
    off = scen.route_off
    first = np.zeros(len(scen.route_links), bool)
    first[off[:-1]] = True
    prev = np.empty_like(exit_t)
    prev[1:] = exit_t[:-1]
    prev[first] = -1
    ok = (~first) & (exit_t >= 0) & (prev >= 0)
    dur = (exit_t - prev)[ok].astype(np.float64)
    links = scen.route_links[ok]
    tot = np.bincount(links, weights=dur, minlength=L)
    cnt = np.bincount(links, minlength=L)
    free = scen.link_len / float(scen.vmax)
    return np.where(cnt > 0, tot / np.maximum(cnt, 1), free)


def reroute(scen, times: np.ndarray, frac: float,
            rng: np.random.Generator):
    """The scenario with a random `frac` of its travellers on the shortest
    path under `times` between their origin and destination.  Returns the
    new scenario and the ids re-routed."""
    n = scen.n_veh
    k = int(round(frac * n))
    ids = np.sort(rng.choice(n, size=k, replace=False)) if k else \
        np.zeros(0, np.int64)
    if k == 0:
        return scen, ids
    off = scen.route_off
    orig = scen.link_from[scen.route_links[off[ids]]]
    dest = scen.link_to[scen.route_links[off[ids + 1] - 1]]
    # integer weights keep Dijkstra's ties deterministic; at least 1
    w = np.maximum(np.rint(times * 16), 1).astype(np.int64)
    new_off, new_links = S.shortest_routes(scen.n_nodes, scen.link_from,
                                           scen.link_to, w, orig, dest)
    lens = np.diff(off).astype(np.int64)
    lens[ids] = np.diff(new_off)
    route_off = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=route_off[1:])
    route_links = np.empty(int(route_off[-1]), np.int32)
    keep = np.ones(n, bool)
    keep[ids] = False
    # copy the kept routes and place the new ones, vehicle by vehicle ranges
    src_starts, dst_starts = off[:-1][keep], route_off[:-1][keep]
    klens = lens[keep]
    rep = np.repeat(np.arange(len(klens)), klens)
    within = np.arange(int(klens.sum())) - np.repeat(np.cumsum(klens) - klens,
                                                    klens)
    route_links[dst_starts[rep] + within] = \
        scen.route_links[src_starts[rep] + within]
    nl = np.diff(new_off)
    rep = np.repeat(np.arange(k), nl)
    within = np.arange(int(nl.sum())) - np.repeat(np.cumsum(nl) - nl, nl)
    route_links[route_off[ids][rep] + within] = new_links
    return dataclasses.replace(scen, route_off=route_off,
                               route_links=route_links), ids


def trip_times(scen, exit_t: np.ndarray) -> np.ndarray:
    """Arrival step - departure step of every traveller that arrived."""
    last = exit_t[scen.route_off[1:] - 1]
    done = last >= 0
    return (last[done] - scen.depart[done]).astype(np.int64)


def run_series(scen, n_runs: int = 50, frac: float = 0.1, seed: int = 7,
               feedback: bool = True, ctx=None, log=None) -> List[Dict]:
    """n_runs micro-simulations with re-routing in between.  Returns one
    record per run (its plans' hash, trip times, timings); the final plans
    are in the last record's "scenario"."""
    import torch
    from .sim import Context
    own = ctx is None
    if own:
        ctx = Context(max_slots=1)
    rng = np.random.Generator(np.random.PCG64(seed))
    costs: Optional[np.ndarray] = None
    out = []
    for r in range(n_runs):
        t0 = time.perf_counter()
        ctx.load(0, scen, link_cost=costs if feedback else None)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.step(0, scen.T)
        st = ctx.stats(0)
        t2 = time.perf_counter()
        exit_t = ctx.state(0)["exit_t"]
        if feedback:
            costs = ctx.link_costs(0)
        tiling = ctx.tiling(0)
        tt = trip_times(scen, exit_t)
        times = link_travel_times(scen, exit_t)
        rec = {"run": r, "hash": st["hash"], "arrived": int(st["n_arrived"]),
               "mean_trip": float(tt.mean()) if len(tt) else float("nan"),
               "veh_updates": int(st["veh_updates"]),
               "gpu_s": t2 - t1, "load_s": t1 - t0,
               "e_tile": tiling["e_tile"], "scenario": scen}
        t3 = time.perf_counter()
        scen, _ = reroute(scen, times, frac, rng)
        rec["reroute_s"] = time.perf_counter() - t3
        out.append(rec)
        if log:
            log(f"run {r}: arrived {rec['arrived']}, mean trip "
                f"{rec['mean_trip']:.1f} s, gpu {rec['gpu_s'] * 1e3:.1f} ms, "
                f"reroute {rec['reroute_s']:.2f} s")
    if own:
        ctx.close()
    return out
