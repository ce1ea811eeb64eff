"""Tiling and launch-shape autotuner for libtransims workloads.

The paper balances load by measuring it: tiles of links are re-weighted by
the time they took in an earlier run (Section "Adaptive Load Balancing").
On the GPU the knobs that decide how a step's work maps onto workgroups are
the tile size (lanes per workgroup), the number of wavefronts that share a
heavy tile in the move sub-step (single scenario only) and the number of
steps per HIP graph replay.  The autotuner times short runs of the real
workload under each candidate, by coordinate descent over the three knobs,
and returns the fastest.  Every candidate must end in the same state (the
trajectory does not depend on the tiling); a candidate that does not is an
error, not a slower option.
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

TILE_LANES = (8, 16, 32, 64)
BACK_PIECES = (1, 2, 4, 8)
GRAPH_STEPS = (32, 64, 128)


def _trial(scens: Sequence, cfg: Dict[str, int], warm_steps: int,
           trial_steps: int, reps: int) -> Dict:
    import torch
    from .sim import Context
    ctx = Context(max_slots=len(scens), tile_lanes=cfg["tile_lanes"],
                  back_pieces=cfg["back_pieces"],
                  graph_steps=cfg["graph_steps"])
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
             graph_steps: Sequence[int] = GRAPH_STEPS, log=None) -> Dict:
    """Times the workload `scens` (all stepped together, as sim_step would
    run them) under candidate configurations and returns the fastest:
    {"tile_lanes", "back_pieces", "graph_steps", "us_per_step", "trials"}.

    Each trial loads every scenario afresh, runs warm_steps steps (so that
    the network holds its mid-run load, not the empty start) and then
    reps x trial_steps timed steps, keeping the best repetition."""
    scens = list(scens)
    if not scens:
        raise ValueError("no scenarios to tune")
    trial_steps = max(1, trial_steps)
    single = len(scens) == 1
    cur = {"tile_lanes": 16, "back_pieces": 4 if single else 1,
           "graph_steps": 64}
    trials: List[Dict] = []
    seen: Dict[tuple, Dict] = {}

    def run(cfg):
        key = (cfg["tile_lanes"], cfg["back_pieces"], cfg["graph_steps"])
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
    if single:
        knobs.append(("back_pieces", back_pieces))
    knobs.append(("graph_steps", graph_steps))
    for name, values in knobs:
        best = None
        for v in values:
            r = run({**cur, name: int(v)})
            if best is None or r["us_per_step"] < best["us_per_step"]:
                best = r
        cur[name] = best[name]
    final = seen[(cur["tile_lanes"], cur["back_pieces"], cur["graph_steps"])]
    return {**cur, "us_per_step": final["us_per_step"],
            "trials": [{k: t[k] for k in ("tile_lanes", "back_pieces",
                                          "graph_steps", "us_per_step")}
                       for t in trials]}
