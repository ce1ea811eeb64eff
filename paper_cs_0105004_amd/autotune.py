"""Tiling and launch-shape autotuner for libtransims workloads.

The paper balances load by measuring it: tiles of links are re-weighted by
the time they took in an earlier run (Section "Adaptive Load Balancing").
On the GPU the knobs that decide how a step's work maps onto workgroups are
the tile size (lanes and cells per workgroup), the number of wavefronts that
share a heavy tile in the move sub-step (single scenario only) and the
number of steps per HIP graph replay.  The autotuner times short runs of
the real workload under each candidate, by coordinate descent over the
knobs, and returns the fastest.  Every candidate must end in the same state (the
trajectory does not depend on the tiling); a candidate that does not is an
error, not a slower option.
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

TILE_LANES = (8, 16, 32, 64)
TILE_CELLS = (1024, 2048, 4096, 6144, 8192, 12288, 16384)
BACK_PIECES = (1, 2, 4, 8)
GRAPH_STEPS = (32, 64, 128)


def _trial(scens: Sequence, cfg: Dict[str, int], warm_steps: int,
           trial_steps: int, reps: int) -> Dict:
    import torch
    from .sim import Context
    ctx = Context(max_slots=len(scens), tile_lanes=cfg["tile_lanes"],
                  back_pieces=cfg["back_pieces"],
                  graph_steps=cfg["graph_steps"],
                  tile_cells=cfg["tile_cells"])
    try:
        slots = list(range(len(scens)))
        for k, sc in enumerate(scens):
            ctx.load(k, sc)
        ctx.step(slots, warm_steps)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            ctx.step(slots, trial_steps)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        hashes = tuple(ctx.stats(k)["hash"] for k in slots)
    finally:
        ctx.close()
    return {**cfg, "us_per_step": best / trial_steps * 1e6, "hashes": hashes}


def autotune(scens: Sequence, warm_steps: int = 600, trial_steps: int = 128,
             reps: int = 2, tile_lanes: Sequence[int] = TILE_LANES,
             back_pieces: Sequence[int] = BACK_PIECES,
             graph_steps: Sequence[int] = GRAPH_STEPS,
             tile_cells: Sequence[int] = TILE_CELLS, log=None) -> Dict:
    """Times the workload `scens` (all stepped together, as sim_step would
    run them) under candidate configurations and returns the fastest:
    {"tile_lanes", "tile_cells", "back_pieces", "graph_steps", "us_per_step",
    "trials"}.  tile_cells only matters for scenarios stepped by one kernel
    per step (no lane changes), back_pieces only for one scenario stepped by
    two kernels; each is tuned only where it can matter.

    Each trial loads every scenario afresh, runs warm_steps steps (so that
    the network holds its mid-run load, not the empty start) and then
    reps x trial_steps timed steps, keeping the best repetition."""
    scens = list(scens)
    if not scens:
        raise ValueError("no scenarios to tune")
    trial_steps = max(1, trial_steps)
    single = len(scens) == 1
    from .scenarios import FLAG_LANE_CHANGE

    def one_kernel(sc):
        return (not (sc.flags & FLAG_LANE_CHANGE)
                and int(sc.link_len.min()) >= 2 * sc.vmax)

    fused = any(one_kernel(sc) for sc in scens if not sc.ring)
    two = any(not one_kernel(sc) for sc in scens if not sc.ring)
    cur = {"tile_lanes": 16, "tile_cells": 2048,
           "back_pieces": 4 if single else 1, "graph_steps": 64}
    trials: List[Dict] = []
    seen: Dict[tuple, Dict] = {}

    def run(cfg):
        key = (cfg["tile_lanes"], cfg["tile_cells"], cfg["back_pieces"],
               cfg["graph_steps"])
        if key not in seen:
            r = _trial(scens, cfg, warm_steps, trial_steps, reps)
            if trials and r["hashes"] != trials[0]["hashes"]:
                raise RuntimeError(f"configuration {key} changed the results")
            seen[key] = r
            trials.append(r)
            if log:
                log(f"autotune {key}: {r['us_per_step']:.2f} us/step")
        return seen[key]

    knobs = [("tile_lanes", tile_lanes)]
    if fused:
        knobs.append(("tile_cells", tile_cells))
    if single and two:
        knobs.append(("back_pieces", back_pieces))
    knobs.append(("graph_steps", graph_steps))
    # coordinate descent, repeated while a pass still moves (at most 3)
    for _ in range(3):
        before = dict(cur)
        for name, values in knobs:
            best = None
            for v in values:
                r = run({**cur, name: int(v)})
                if best is None or r["us_per_step"] < best["us_per_step"]:
                    best = r
            cur[name] = best[name]
        if cur == before:
            break
    final = seen[(cur["tile_lanes"], cur["tile_cells"], cur["back_pieces"],
                  cur["graph_steps"])]
    return {**cur, "us_per_step": final["us_per_step"],
            "trials": [{k: t[k] for k in ("tile_lanes", "tile_cells",
                                          "back_pieces", "graph_steps",
                                          "us_per_step")}
                       for t in trials]}
