"""Host side of the iteration series: link travel times from exit times,
the re-routing of a fraction of the travellers, and the whole loop with the
oracle standing in for the GPU context."""
import numpy as np

from paper_cs_0105004_amd import iteration as I
from paper_cs_0105004_amd import scenarios as S


def test_link_travel_times_by_hand():
    scen = S.chain([10, 12, 14], depart=(0, 2), vmax=5, T=50)
    # vehicle 0 left links 0,1,2 in steps 3, 6, 10; vehicle 1 left link 0 in
    # step 5 and link 1 in step 11, and is still on link 2
    exit_t = np.array([3, 6, 10, 5, 11, -1], np.int32)
    t = I.link_travel_times(scen, exit_t)
    assert t[0] == 10 / 5          # first links do not count: free flow
    assert t[1] == (3 + 6) / 2     # 6-3 and 11-5
    assert t[2] == 4               # 10-6; vehicle 1 has not left link 2


def test_reroute_keeps_endpoints_and_connectivity():
    scen = S.portland_like(scale=0.05, T=100)
    rng = np.random.Generator(np.random.PCG64(3))
    times = rng.uniform(1, 50, scen.n_links)
    new, ids = I.reroute(scen, times, 0.1,
                         np.random.Generator(np.random.PCG64(4)))
    assert len(ids) == round(0.1 * scen.n_veh)
    o0, o1 = scen.route_off, new.route_off
    moved = np.zeros(scen.n_veh, bool)
    moved[ids] = True
    for i in range(scen.n_veh):
        a = scen.route_links[o0[i]:o0[i + 1]]
        b = new.route_links[o1[i]:o1[i + 1]]
        assert scen.link_from[a[0]] == new.link_from[b[0]]
        assert scen.link_to[a[-1]] == new.link_to[b[-1]]
        assert (new.link_to[b[:-1]] == new.link_from[b[1:]]).all()
        if not moved[i]:
            assert np.array_equal(a, b)
    # the re-routed travellers follow the cheaper paths under `times`
    cost = lambda sc, i: times[sc.route_links[sc.route_off[i]:
                                              sc.route_off[i + 1]]].sum()
    assert sum(cost(new, i) for i in ids) <= sum(cost(scen, i) for i in ids)
    # deterministic for a seed
    again, ids2 = I.reroute(scen, times, 0.1,
                            np.random.Generator(np.random.PCG64(4)))
    assert np.array_equal(ids, ids2)
    assert np.array_equal(again.route_links, new.route_links)


def test_series_loop_on_the_oracle(monkeypatch):
    # the whole loop with the oracle standing in for the GPU context: each
    # run simulates the current plans, and re-routing changes the plans of
    # about the stated fraction of travellers and nothing else
    import torch

    import oracle
    from paper_cs_0105004_amd import iteration as It
    from paper_cs_0105004_amd import sim

    class OracleContext:
        def __init__(self, max_slots=1, **kw):
            self.o = None

        def load(self, k, scen, link_cost=None):
            if self.o:
                self.o.close()
            self.o = oracle.OracleSim(scen)

        def step(self, k, n):
            self.o.step(n)

        def stats(self, k):
            return self.o.stats()

        def state(self, k):
            return self.o.state()

        def tiling(self, k):
            return {"e_tile": 1.0}

        def link_costs(self, k):
            raise AssertionError("no feedback was asked for")

        def close(self):
            self.o.close()

    monkeypatch.setattr(sim, "Context", OracleContext)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a: None)
    scen = S.portland_like(scale=0.02, T=300, depart_max=100, seed=4)
    recs = It.run_series(scen, n_runs=3, frac=0.2, seed=1, feedback=False)
    assert [r["run"] for r in recs] == [0, 1, 2]
    for r in recs:
        o = oracle.OracleSim(r["scenario"])
        o.step(r["scenario"].T)
        assert r["hash"] == o.stats()["hash"]
        o.close()
    a, b = recs[0]["scenario"], recs[1]["scenario"]
    changed = sum(not np.array_equal(
        a.route_links[a.route_off[i]:a.route_off[i + 1]],
        b.route_links[b.route_off[i]:b.route_off[i + 1]]) for i in range(a.n_veh))
    assert 0 < changed <= round(0.2 * a.n_veh)
