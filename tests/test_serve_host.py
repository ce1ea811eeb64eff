"""The serving loop's scheduling on the CPU, with a stand-in for the
libtransims context that records what it is asked to do: FIFO admission
under the memory budget and the slot count, every run stepped exactly to
its horizon in shared chunks, slots and memory given back, and the
latency summary."""
import types

import numpy as np
import pytest

from paper_cs_0105004_amd import serve


class FakeContext:
    def __init__(self, max_slots, sizes):
        self.max_slots, self.sizes = max_slots, sizes
        self.loaded, self.steps, self.log = {}, {}, []
        self.stream = None

    def footprint(self, scen):
        return self.sizes[scen.key]

    def load(self, slot, scen):
        assert slot not in self.loaded and 0 <= slot < self.max_slots
        self.loaded[slot] = scen
        self.steps[slot] = 0
        self.log.append(("load", slot, scen.key))

    def step(self, slots, n):
        assert len(set(slots)) == len(slots) and n > 0
        for s in slots:
            assert s in self.loaded
            self.steps[s] += n
        self.log.append(("step", tuple(slots), n))

    def stats(self, slot):
        return {"veh_updates": 10 * self.steps[slot], "t": self.steps[slot]}

    def state(self, slot):
        return {"exit_t": np.full(3, self.steps[slot], np.int32)}

    def unload(self, slot):
        self.log.append(("unload", slot, self.steps.pop(slot)))
        del self.loaded[slot]

    def close(self):
        pass


class FakeEvent:
    def record(self, stream):
        pass

    def synchronize(self):
        pass


def server(max_slots, budget, sizes, chunk, background=False):
    srv = object.__new__(serve.Server)  # no GPU: the constructor is bypassed
    srv.torch = types.SimpleNamespace(cuda=types.SimpleNamespace(
        Event=FakeEvent, set_device=lambda d: None))
    srv.device = 0
    srv.ctx = FakeContext(max_slots, sizes)
    srv.budget, srv.max_slots, srv.chunk = budget, max_slots, chunk
    srv.read_exit_times, srv.log = True, []
    srv.background = background
    return srv


def scen(key, T):
    return types.SimpleNamespace(key=key, T=T)


def test_admission_budget_fifo_and_horizons():
    rng = np.random.default_rng(5)
    sizes = {k: int(s) for k, s in enumerate(rng.integers(10, 60, size=12))}
    pool = [scen(k, int(rng.integers(1, 300))) for k in range(12)]
    reqs = [serve.Request(i, 0.0, pool[int(rng.integers(12))]) for i in range(40)]
    srv = server(max_slots=4, budget=120, sizes=sizes, chunk=64)
    res = srv.run(reqs, realtime=False)
    assert sorted(r.rid for r in res) == list(range(40))
    used, loaded, order = 0, {}, []
    for ev in srv.ctx.log:
        if ev[0] == "load":
            loaded[ev[1]] = ev[2]
            used += sizes[ev[2]]
            order.append(ev[2])
            assert used <= 120 and len(loaded) <= 4
        elif ev[0] == "unload":
            used -= sizes[loaded.pop(ev[1])]
        else:
            assert all(s in loaded for s in ev[1]) and ev[2] <= 64
    assert used == 0 and not loaded
    # admission is first come, first served
    assert order == [r.scen.key for r in reqs]
    # every run was stepped exactly to its horizon
    for r in res:
        assert r.stats["t"] == reqs[r.rid].scen.T
        assert (r.exit_t == r.stats["t"]).all()
        assert r.admitted_s >= r.arrival_s and r.done_s >= r.admitted_s


def test_runs_share_chunks():
    sizes = {0: 10, 1: 10}
    reqs = [serve.Request(0, 0.0, scen(0, 100)), serve.Request(1, 0.0, scen(1, 130))]
    srv = server(max_slots=2, budget=100, sizes=sizes, chunk=64)
    srv.run(reqs, realtime=False)
    steps = [ev for ev in srv.ctx.log if ev[0] == "step"]
    # both runs advance in the same calls until the shorter one ends
    assert steps[0] == ("step", (0, 1), 64)
    assert steps[1] == ("step", (0, 1), 36)
    assert steps[2][1] == (1,) and sum(e[2] for e in steps[2:]) == 30


def test_request_larger_than_the_budget():
    srv = server(max_slots=2, budget=50, sizes={0: 51}, chunk=8)
    with pytest.raises(RuntimeError, match="budget"):
        srv.run([serve.Request(0, 0.0, scen(0, 5))], realtime=False)


def test_summary_percentiles():
    res = [serve.Result(i, 0.0, 0.0, float(i + 1), {"veh_updates": 100}, None, 1)
           for i in range(100)]
    out = serve.summarize(res, wall_s=2.0)
    assert out["requests"] == 100 and out["vehicle_updates"] == 10000
    assert out["updates_per_s"] == 5000.0
    assert out["p50_latency_s"] in (50.0, 51.0)
    assert out["p99_latency_s"] == 99.0 and out["max_latency_s"] == 100.0
    assert serve.percentile([], 0.5) != serve.percentile([], 0.5)  # nan


class SlowLoadContext(FakeContext):
    """Loads block until the driving thread has stepped the runs already
    loaded a given number of times (or nothing else runs)."""

    def __init__(self, max_slots, sizes, steps_before_load):
        super().__init__(max_slots, sizes)
        import threading
        self.cv = threading.Condition()
        self.n_steps = 0
        self.wait_for = steps_before_load

    def load(self, slot, scen):
        with self.cv:
            self.cv.wait_for(lambda: self.n_steps >= self.wait_for
                             or not self.loaded, timeout=5.0)
            super().load(slot, scen)

    def step(self, slots, n):
        with self.cv:
            super().step(slots, n)
            self.n_steps += 1
            self.cv.notify_all()


def test_background_loads_keep_the_running_slots_stepping():
    sizes = {0: 10, 1: 10, 2: 10}
    reqs = [serve.Request(0, 0.0, scen(0, 640)),
            serve.Request(1, 0.0, scen(1, 100)),
            serve.Request(2, 0.0, scen(2, 50))]
    srv = server(max_slots=3, budget=100, sizes=sizes, chunk=64,
                 background=True)
    srv.ctx = SlowLoadContext(3, sizes, steps_before_load=3)
    res = srv.run(reqs, realtime=False)
    assert sorted(r.rid for r in res) == [0, 1, 2]
    for r in res:
        assert r.stats["t"] == reqs[r.rid].scen.T
    log = srv.ctx.log
    # the first run was stepped while the others were still loading
    first_other = min(i for i, ev in enumerate(log)
                      if ev[0] == "load" and ev[2] != 0)
    assert sum(1 for ev in log[:first_other] if ev[0] == "step") >= 3
    assert [ev for ev in log if ev[0] == "unload"] and not srv.ctx.loaded
