"""Edge cases of the network step on the GPU, in both step modes, against
the CPU oracle: extreme speeds and slowdown probabilities, every vehicle
departing at once, four lanes everywhere, the longest links the library
accepts (also with lane changes, whose bit lattice of a 4-lane link of
32,767 cells takes 4,096 words of LDS), the smallest grid, and a scenario
with no vehicles at all."""
import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S
from parity import assert_same_state, assert_same_stats, run_side_by_side

pytestmark = pytest.mark.gpu


def _ctx(mode, **kw):
    from paper_cs_0105004_amd.sim import Context
    return Context(max_slots=1, step_mode=mode, **kw)


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("vmax,p", [(1, "0"), (1, "1"), (3, "0.5"),
                                    (7, "0"), (7, "0.2"), (5, "1")])
def test_speed_and_slowdown_extremes(mode, vmax, p):
    scen = S.grid_scenario(6, 7, 100, 400, T=250, depart_max=100, seed=11,
                           vmax=vmax, p=p)
    ctx = _ctx(mode)
    o = run_side_by_side(ctx, 0, scen, 250, every=50, full_at=(100,))
    if p == "1":  # from rest nobody ever accelerates past 0
        assert o.stats()["sum_v"] == 0
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_everyone_departs_at_once(mode):
    # long parking queues on every origin link, all released at t = 0
    scen = S.grid_scenario(5, 5, 64, 3000, T=300, depart_max=0, seed=12)
    ctx = _ctx(mode)
    run_side_by_side(ctx, 0, scen, 300, every=30, full_at=(1, 2, 150))
    ctx.close()


@pytest.mark.parametrize("mode,flags", [
    (0, 0), (1, 0), (1, S.FLAG_LANE_CHANGE),
    (1, S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES)])
def test_four_lanes_everywhere(mode, flags):
    scen = S.grid_scenario(5, 6, 80, 1500, T=300, depart_max=120, seed=13,
                           lanes_range=(4, 4), flags=flags)
    ctx = _ctx(mode)
    o = run_side_by_side(ctx, 0, scen, 300, every=60, full_at=(120,))
    if flags & S.FLAG_LANE_CHANGE:
        assert o.stats()["lane_changes"] > 0
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_longest_links(mode):
    # 32,767 cells is the largest link length the library takes
    def lengths(rng, m):
        return rng.integers(30000, 32768, size=m)
    scen = S.grid_scenario(3, 3, 16, 60, T=200, depart_max=50, seed=14,
                           len_sampler=lengths)
    assert scen.link_len.max() <= 32767
    ctx = _ctx(mode)
    run_side_by_side(ctx, 0, scen, 200, every=100)
    ctx.close()


@pytest.mark.parametrize("tile_cells", [0, 64])
def test_lane_changes_on_the_longest_links(tile_cells):
    # 4-lane links of 30,000-32,767 cells with lane changes and turn lanes:
    # each tile holds one link (tile_cells caps the tiles in cells)
    def lengths(rng, m):
        return rng.integers(30000, 32768, size=m)
    scen = S.grid_scenario(3, 3, 16, 400, T=150, depart_max=40, seed=17,
                           len_sampler=lengths, lanes_range=(4, 4),
                           flags=S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES)
    ctx = _ctx(1, tile_cells=tile_cells)
    o = run_side_by_side(ctx, 0, scen, 150, every=50, full_at=(75,))
    assert o.stats()["lane_changes"] > 0
    ctx.close()


@pytest.mark.parametrize("tile_lanes,p_lc", [(64, "1"), (8, "1"), (64, "0.6")])
def test_lane_changes_in_a_jam(tile_lanes, p_lc):
    # every vehicle released at t = 0 onto short 2-4 lane links: many
    # vehicles per tile (several batches of the lane-change pass); with
    # p_lc < 1 every discretionary change takes a draw, which needs the
    # vehicle's id from its record in every batch
    scen = S.grid_scenario(4, 5, 40, 6000, T=200, depart_max=0, seed=18,
                           lanes_range=(2, 4),
                           flags=S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES)
    scen.lc_thr = S.prob_threshold(p_lc)
    ctx = _ctx(1, tile_lanes=tile_lanes, tile_cells=65536)
    o = run_side_by_side(ctx, 0, scen, 200, every=20, full_at=(1, 2, 100))
    assert o.stats()["lane_changes"] > 0
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_smallest_grid_with_one_tile_per_lane(mode):
    scen = S.grid_scenario(2, 2, 8, 30, T=300, depart_max=40, seed=15)
    ctx = _ctx(mode, tile_lanes=1, tile_cells=64)
    run_side_by_side(ctx, 0, scen, 300, every=1, full_at=(10, 100, 200))
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_no_vehicles(mode):
    scen = S.grid_scenario(3, 4, 22, 0, T=50, depart_max=10, seed=16)
    assert scen.n_veh == 0
    ctx = _ctx(mode)
    ctx.load(0, scen)
    ctx.step(0, 50)
    st = ctx.stats(0)
    o = oracle.OracleSim(scen)
    o.step(50)
    assert_same_stats(st, o.stats(), "empty")
    assert st["veh_updates"] == 0 and st["n_active"] == 0
    g = ctx.state(0)
    assert all(len(g[k]) == 0 for k in ("status", "x", "exit_t"))
    ctx.close()


def test_batched_lane_change_slots_with_different_lattices():
    # three lane-changing scenarios stepped in the same launches: the launch
    # reserves LDS for the largest lattice (4-lane links of ~15k cells), each
    # slot's tiles use their own part of it
    def lengths(rng, m):
        return rng.integers(14000, 16001, size=m)
    flags = S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES
    scens = [
        S.grid_scenario(3, 3, 16, 300, T=200, depart_max=40, seed=19,
                        len_sampler=lengths, lanes_range=(4, 4), flags=flags),
        S.portland_like(scale=0.01, T=200, depart_max=100, seed=51,
                        flags=flags),
        S.grid_scenario(4, 5, 40, 3000, T=200, depart_max=0, seed=52,
                        lanes_range=(2, 4), flags=flags),
    ]
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=len(scens))
    for k, sc in enumerate(scens):
        ctx.load(k, sc)
    ctx.step([0, 1, 2], 150)
    ctx.step([0, 2], 30)  # uneven progress
    steps = [180, 150, 180]
    for k, sc in enumerate(scens):
        o = oracle.OracleSim(sc)
        o.step(steps[k])
        assert_same_stats(ctx.stats(k), o.stats(), f"slot {k}")
        assert_same_state(ctx.state(k), o.state(), f"slot {k}")
        assert o.stats()["lane_changes"] > 0
    ctx.close()


def test_lane_change_tiles_reordered_between_graph_replays():
    # one link per tile, three lane-changing slots in one list: between
    # 6,144 and 16,384 tiles, so every graph replay first reorders each
    # XCD's tiles by the time each took in the lane-change kernel since the
    # replay before (entries of different slots mixed); the order changes
    # no result
    flags = S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES
    scens = [S.portland_like(scale=sc, T=200, depart_max=100, seed=sd,
                             flags=flags)
             for sc, sd in ((0.15, 62), (0.1, 61), (0.15, 63))]
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=len(scens), tile_lanes=1, tile_cells=64,
                  graph_steps=32)
    for k, sc in enumerate(scens):
        ctx.load(k, sc)
    ctx.step([0, 1, 2], 192)  # six replays
    n_tiles = sum(ctx.tiling(k)["n_tiles"] for k in range(len(scens)))
    assert 6144 < n_tiles <= 8 * 2048, n_tiles
    for k, sc in enumerate(scens):
        o = oracle.OracleSim(sc)
        o.step(192)
        assert_same_stats(ctx.stats(k), o.stats(), f"slot {k}")
        assert_same_state(ctx.state(k), o.state(), f"slot {k}")
        assert o.stats()["lane_changes"] > 0
    ctx.close()
