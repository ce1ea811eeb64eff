"""Serving loop: scenario runs admitted by HBM footprint and stepped together.

The paper's production use is a series of about fifty simulation runs, fed
back through the router between runs (Section "Introduction"; Section
"Other modules"), so what matters is the throughput of many runs, not one.
Here runs arrive as requests.  The loop:

* admits arrived requests in FIFO order while a slot is free and the
  request's workspace (sim_footprint) fits the remaining HBM budget; the
  admitted request is loaded by a loader thread (the library allows loads
  on another thread for slots no concurrent call names), so the runs
  already on the device keep stepping while its network and routes are
  checked, encoded and copied;
* advances every admitted run together, `chunk` steps per sim_step call
  (continuous batching: a request that arrives while others run joins the
  next chunk, and all of them share the same kernel launches);
* retires a run when it reaches its horizon: its statistics and per-route
  exit times are read back, its slot and workspace are released, and the
  completion latency (result available minus arrival) is recorded.

A run's results do not depend on which other runs share its launches: the
update of a scenario reads only its own state and its own counter-based
draws.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time
from typing import Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float  # seconds after the start of the trace
    scen: object      # a scenarios.Scenario; its T is the horizon


@dataclasses.dataclass
class Result:
    rid: int
    arrival_s: float
    admitted_s: float
    done_s: float
    stats: Dict
    exit_t: np.ndarray
    footprint: int

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def poisson_trace(pool: Sequence, rate_per_s: float, window_s: float,
                  seed: int = 9) -> List[Request]:
    """Poisson arrivals at `rate_per_s` over `window_s` seconds, each
    request drawing one (network, demand) set of `pool` at random."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate_per_s))
        if t > window_s:
            return out
        out.append(Request(len(out), t, pool[int(rng.integers(len(pool)))]))


def percentile(xs: Sequence[float], q: float) -> float:
    s = sorted(xs)
    if not s:
        return float("nan")
    return s[min(len(s) - 1, int(round(q * (len(s) - 1))))]


class Server:
    """A continuous-batching loop over one libtransims context."""

    def __init__(self, max_slots: int = 64, budget_bytes: Optional[int] = None,
                 chunk: int = 64, tile_lanes: int = 0, graph_steps: int = 0,
                 read_exit_times: bool = True, background_loads: bool = True):
        import torch
        from .sim import Context
        self.torch = torch
        self.ctx = Context(max_slots=max_slots, tile_lanes=tile_lanes,
                           graph_steps=graph_steps)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.chunk = max(1, int(chunk))
        self.read_exit_times = read_exit_times
        self.background = background_loads
        self.device = torch.cuda.current_device()
        self.log: List[str] = []

    def close(self):
        self.ctx.close()

    def run(self, requests: Sequence[Request], realtime: bool = True
            ) -> List[Result]:
        """Serves `requests` (sorted by arrival).  With realtime, a request
        becomes visible when the wall clock since the start passes its
        arrival time; otherwise every request is visible at once."""
        future = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        pending: collections.deque = collections.deque()
        free_slots = list(range(self.max_slots - 1, -1, -1))
        active: Dict[int, list] = {}  # slot -> [request, steps left, bytes, admitted]
        loading: Dict[int, list] = {}  # slot -> [request, bytes, admitted]
        used = 0
        results: List[Result] = []
        fp_cache: Dict[int, int] = {}
        inflight: collections.deque = collections.deque()  # chunk events
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        jobs: queue.Queue = queue.Queue()
        done: queue.Queue = queue.Queue()

        def loader():
            setup = None
            try:
                self.torch.cuda.set_device(self.device)
            except BaseException as e:  # reported with the first job
                setup = e
            while True:
                job = jobs.get()
                if job is None:
                    return
                slot, r = job
                try:
                    if setup is not None:
                        raise setup
                    self.ctx.load(slot, r.scen)
                    done.put((slot, None))
                except BaseException as e:  # handed to the driving thread
                    done.put((slot, e))

        def loaded(item):
            slot, err = item
            if err is not None:
                raise err
            r, fp, adm = loading.pop(slot)
            active[slot] = [r, int(r.scen.T), fp, adm]

        th = None
        if self.background:
            th = threading.Thread(target=loader, daemon=True)
            th.start()
        try:
            while future or pending or active or loading:
                tn = now()
                while future and (not realtime or future[0].arrival_s <= tn):
                    pending.append(future.popleft())
                # admission, FIFO: the head waits until it fits
                while pending and free_slots:
                    r = pending[0]
                    key = id(r.scen)
                    if key not in fp_cache:
                        fp_cache[key] = self.ctx.footprint(r.scen)
                    fp = fp_cache[key]
                    if fp > self.budget:
                        raise RuntimeError(f"request {r.rid} needs {fp} bytes, "
                                           f"more than the budget {self.budget}")
                    if used + fp > self.budget:
                        break
                    slot = free_slots.pop()
                    used += fp
                    loading[slot] = [r, fp, now()]
                    pending.popleft()
                    if self.background:
                        jobs.put((slot, r))
                    else:
                        self.ctx.load(slot, r.scen)
                        loaded((slot, None))
                # loads that finished join the batch at this chunk boundary
                while True:
                    try:
                        loaded(done.get_nowait())
                    except queue.Empty:
                        break
                if not active:
                    if loading:
                        # nothing to step: wait for a load (or the next
                        # arrival, which may be admitted meanwhile)
                        wait = None
                        if future and realtime:
                            wait = max(0.0, future[0].arrival_s - now())
                        try:
                            loaded(done.get(timeout=wait))
                        except queue.Empty:
                            pass
                    elif future and realtime:
                        time.sleep(max(0.0, future[0].arrival_s - now()))
                    continue
                slots = sorted(active)
                n = min(self.chunk, min(active[s][1] for s in slots))
                if n > 0:
                    self.ctx.step(slots, n)
                    # keep the host at most two chunks ahead of the device,
                    # so that arrivals are admitted at the next chunk
                    # boundary
                    ev = self.torch.cuda.Event()
                    ev.record(self.ctx.stream)
                    inflight.append(ev)
                    while len(inflight) > 2:
                        inflight.popleft().synchronize()
                for s in slots:
                    active[s][1] -= n
                for s in [s for s in slots if active[s][1] <= 0]:
                    r, _, fp, adm = active.pop(s)
                    st = self.ctx.stats(s)
                    ex = (self.ctx.state(s)["exit_t"] if self.read_exit_times
                          else np.zeros(0, np.int32))
                    results.append(Result(r.rid, r.arrival_s, adm, now(), st,
                                          ex, fp))
                    self.ctx.unload(s)
                    used -= fp
                    free_slots.append(s)
        finally:
            if th is not None:
                jobs.put(None)
                th.join()
        return results


def summarize(results: Sequence[Result], wall_s: float) -> Dict:
    lat = [r.latency_s for r in results]
    upd = sum(r.stats["veh_updates"] for r in results)
    return {"requests": len(results), "vehicle_updates": upd,
            "wall_s": wall_s, "updates_per_s": upd / wall_s if wall_s else 0.0,
            "p50_latency_s": percentile(lat, 0.5),
            "p99_latency_s": percentile(lat, 0.99),
            "max_latency_s": max(lat) if lat else float("nan")}
