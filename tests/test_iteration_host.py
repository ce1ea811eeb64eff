"""Host side of the iteration series: link travel times from exit times and
the re-routing of a fraction of the travellers."""
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
