"""GPU parity: libtransims (through its C ABI) against the CPU oracle, bit
for bit, on the same seeded inputs.  Every step is integer, so the bar is
exact equality of every vehicle's state, every exit time and every counter."""

import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S

from hand_cases import BOUNDARIES, build, check, load_cases
from parity import assert_same_state, assert_same_stats, run_side_by_side

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sim():
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=8)
    yield ctx
    ctx.close()


def test_c1_ring_full_run(sim):
    scen = S.ring()  # 1000 cells, 150 vehicles, vmax 5, p 0.2, seed 42
    run_side_by_side(sim, 0, scen, 1000, every=100, full_at=(1, 2, 10))


@pytest.mark.parametrize("p,vmax", [("0", 5), ("1", 5), ("0.5", 1),
                                    ("0.2", 7)])
def test_ring_variants(sim, p, vmax):
    scen = S.ring(1000, 150, vmax, p=p, seed=42)
    run_side_by_side(sim, 0, scen, 300, every=50)


def test_ring_edge_cases(sim):
    cases = [S.ring(1, 1, 5, "0.3", seed=3), S.ring(7, 0, 5, "0.3"),
             S.ring(5, 5, 3, "0.3"), S.ring(9, 1, 7, "0.5", seed=9),
             S.ring(4096, 4096, 5, "0.2"), S.ring(20000, 4096, 5, "0.2"),
             S.ring(300, 299, 2, "0.1", seed=77)]
    for scen in cases:
        print("case", scen.link_len[0], scen.n_veh, scen.vmax, flush=True)
        run_side_by_side(sim, 1, scen, 40, every=10)


def test_many_rings_in_one_launch(sim):
    scens = [S.ring(int(L), int(n), 5, "0.25", seed=100 + k, placement_seed=k)
             for k, (L, n) in enumerate([(50, 10), (1000, 150), (333, 300),
                                         (2, 1), (700, 0), (4000, 1000)])]
    for k, sc in enumerate(scens):
        sim.load(k, sc)
    sim.step(list(range(len(scens))), 123)
    for k, sc in enumerate(scens):
        o = oracle.OracleSim(sc)
        o.step(123)
        assert_same_stats(sim.stats(k), o.stats(), f"ring {k}")
        assert_same_state(sim.state(k), o.state(), f"ring {k}")


@pytest.fixture(scope="module")
def sim_two_kernel():
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=1, step_mode=1)
    yield ctx
    ctx.close()


@pytest.fixture(scope="module")
def sim_skip():
    # one kernel per step, skipping lanes that are empty and stay empty
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=2, step_mode=2)
    yield ctx
    ctx.close()


# the worked cases and the cases on either side of each comparison of the
# lane-change and node rules, in both step forms; each is checked against
# its hand-worked outcome and against the oracle's complete state
@pytest.mark.parametrize("mode", [0, 1, 2],
                         ids=["one_kernel", "two_kernel", "skip_idle"])
@pytest.mark.parametrize("case", load_cases() + load_cases(BOUNDARIES),
                         ids=lambda c: c["name"])
def test_hand_worked_cases(sim, sim_two_kernel, sim_skip, case, mode):
    ctx = (sim, sim_two_kernel, sim_skip)[mode]
    scen = build(case)
    print("case", case["name"], "mode", mode, flush=True)
    ctx.load(0, scen)
    ctx.step(0, case["steps"])
    g, gs = ctx.state(0), ctx.stats(0)
    check(case, g, gs)
    o = oracle.OracleSim(scen)
    o.step(case["steps"])
    assert_same_stats(gs, o.stats(), case["name"])
    assert_same_state(g, o.state(), case["name"])


@pytest.mark.parametrize("p", ["0", "0.2"])
def test_loop_of_links(sim, p):
    scen = S.loop_of_links([12, 30, 9, 41, 6], 40, vmax=5, p=p, seed=5, T=200)
    run_side_by_side(sim, 0, scen, 200, every=1, full_at=(1, 50))


def small_grid(flags=0, scale=0.01, depart_max=150, seed=2024):
    scen = S.portland_like(scale=scale, T=400, depart_max=depart_max,
                           seed=seed, flags=flags)
    if flags & S.FLAG_TURN_LANES:
        scen.conn_off, scen.conn_out, scen.conn_lo, scen.conn_hi = \
            S._ranks_and_conn(scen.n_nodes, scen.link_from, scen.link_to,
                              scen.link_lanes, scen.node_xy, True)[1:]
    return scen


def test_small_grid_every_step(sim):
    run_side_by_side(sim, 0, small_grid(), 400, every=1,
                     full_at=(1, 2, 3, 50, 100, 200, 300))


@pytest.mark.parametrize("flags", [S.FLAG_LANE_CHANGE,
                                   S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES])
def test_small_grid_lane_change(sim, flags):
    scen = small_grid(flags)
    orc = run_side_by_side(sim, 0, scen, 400, every=1,
                           full_at=(1, 2, 50, 150, 300))
    assert orc.stats()["lane_changes"] > 0


def test_lane_change_slowdown_draws(sim):
    scen = small_grid(S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES)
    scen.lc_thr = S.prob_threshold("0.6")
    run_side_by_side(sim, 0, scen, 300, every=25)


@pytest.mark.parametrize("tile_lanes,pieces,graph",
                         [(1, 1, -1), (4, 8, 5), (37, 3, 1), (64, 8, 64),
                          (16, 4, 64), (16, 1, 7)])
def test_tile_size_does_not_change_results(tile_lanes, pieces, graph):
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=1, tile_lanes=tile_lanes, back_pieces=pieces,
                  graph_steps=graph)
    try:
        run_side_by_side(ctx, 0, small_grid(S.FLAG_LANE_CHANGE, seed=7), 250,
                         every=50)
    finally:
        ctx.close()


def test_medium_grid_ragged_tiles(sim):
    scen = S.portland_like(scale=0.06, T=500, depart_max=400, seed=11)
    run_side_by_side(sim, 0, scen, 500, every=100, full_at=(250,))


def test_skip_idle_batched_slots_come_and_go():
    """Idle-lane skipping with slots loaded and unloaded between calls and
    uneven progress: every slot equals the oracle (a restart from a saved
    state begins with a step that looks at every lane)."""
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=3, step_mode=2, tile_lanes=1)
    a = S.portland_like(scale=0.05, T=900, depart_max=600, seed=21)
    b = S.portland_like(scale=0.2, T=900, depart_max=600, seed=22)
    oa, ob = oracle.OracleSim(a), oracle.OracleSim(b)
    ctx.load(0, a)
    ctx.step(0, 101)
    oa.step(101)
    ctx.load(1, b)
    ctx.step([0, 1], 250)
    oa.step(250)
    ob.step(250)
    assert_same_stats(ctx.stats(1), ob.stats(), "b at 250")
    mid = ctx.state(0)
    ctx.unload(0)
    ctx.load(2, a.with_state(mid, 351))
    ctx.step(2, 77)
    oa.step(77)
    ctx.step([1, 2], 300)
    oa.step(300)
    ob.step(300)
    # (the restarted slot's counters start again at its restart)
    assert ctx.stats(2)["hash"] == oa.stats()["hash"]
    assert_same_state(ctx.state(2), oa.state(), "a")
    assert_same_state(ctx.state(1), ob.state(), "b")
    ctx.close()


def test_batched_slots_equal_solo(sim):
    scens = [small_grid(seed=31), small_grid(S.FLAG_LANE_CHANGE, seed=32),
             S.loop_of_links([12, 30, 9], 20, p="0.3", seed=3, T=300),
             S.ring(500, 80, 5, "0.2", seed=33)]
    for k, sc in enumerate(scens):
        sim.load(k, sc)
    sim.step(list(range(len(scens))), 150)
    sim.step([1, 3], 50)  # uneven progress
    steps = [150, 200, 150, 200]
    for k, sc in enumerate(scens):
        o = oracle.OracleSim(sc)
        o.step(steps[k])
        assert_same_stats(sim.stats(k), o.stats(), f"slot {k}")
        assert_same_state(sim.state(k), o.state(), f"slot {k}")


def test_restart_from_saved_state(sim):
    scen = small_grid(S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES, seed=41)
    sim.load(0, scen)
    sim.step(0, 170)
    mid = sim.state(0)
    sim.step(0, 100)
    end = sim.state(0)
    sim.load(1, scen.with_state(mid, 170))
    sim.step(1, 100)
    assert_same_state(sim.state(1), end, "restart")
    o = oracle.OracleSim(scen)
    o.step(270)
    assert_same_state(end, o.state(), "restart vs oracle")


@pytest.mark.parametrize("tile_lanes,pieces,flags", [(64, 1, 0), (64, 1, S.FLAG_LANE_CHANGE),
                                                     (16, 4, 0), (3, 2, S.FLAG_LANE_CHANGE)])
def test_dense_lanes_many_vehicle_groups(tile_lanes, pieces, flags):
    # lanes holding hundreds of vehicles: one wavefront updates them in many
    # groups of 64, rear first, so every vehicle must still see the old
    # position of the one ahead
    from paper_cs_0105004_amd.sim import Context
    scen = S.loop_of_links([700, 650, 900], 450, vmax=5, p="0.25", seed=9,
                           T=120, lanes=3, placement_seed=4, flags=flags)
    ctx = Context(max_slots=1, tile_lanes=tile_lanes, back_pieces=pieces)
    try:
        run_side_by_side(ctx, 0, scen, 120, every=20, full_at=(1, 60))
    finally:
        ctx.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_step_modes_agree_with_oracle(mode):
    # mode 0 runs this scenario (no lane changes, links >= 2 vmax cells) with
    # one kernel per step, mode 1 with the lane-change and move kernels,
    # mode 2 with one kernel that skips idle lanes
    from paper_cs_0105004_amd.sim import Context
    scen = S.portland_like(scale=0.02, T=400)
    assert scen.link_len.min() >= 2 * scen.vmax
    ctx = Context(max_slots=1, step_mode=mode)
    ctx.profile(True)
    run_side_by_side(ctx, 0, scen, 400, every=40, full_at=(200,))
    kt = ctx.kernel_times()
    if mode != 1:
        assert kt["step"][0] == 400 and kt["front"][0] == 0
    else:
        assert kt["step"][0] == 0 and kt["front"][0] == 400
    ctx.close()


@pytest.mark.parametrize("mode", [0, 2])
def test_one_kernel_step_with_graphs_and_restart(mode):
    from paper_cs_0105004_amd.sim import Context
    scen = S.portland_like(scale=0.05, T=600)
    a = Context(max_slots=2, graph_steps=32, step_mode=mode)
    a.load(0, scen)
    a.step(0, 333)
    mid = a.state(0)
    a.step(0, 267)
    o = oracle.OracleSim(scen)
    o.step(600)
    assert_same_stats(a.stats(0), o.stats(), "graphs")
    assert_same_state(a.state(0), o.state(), "graphs")
    # restart at an odd step: the parity buffers start from the other half
    a.load(1, scen.with_state(mid, 333))
    a.step(1, 267)
    assert_same_state(a.state(1), o.state(), "restart at t=333")
    a.close()


def test_remainder_graphs_reused_and_rebuilt():
    """Calls of fewer steps than a graph replay run as a cached graph of
    their own length: repeated windows reuse it, another length rebuilds it,
    and a remainder below the graph threshold is launched kernel by kernel.
    Every stretch equals the oracle."""
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=1, graph_steps=64)
    scen = S.portland_like(scale=0.02, T=600, depart_max=300, seed=31)
    ctx.load(0, scen)
    o = oracle.OracleSim(scen)
    for n in (20, 20, 20, 30, 5, 64 + 20, 20, 9, 9):
        ctx.step(0, n)
        o.step(n)
        assert_same_stats(ctx.stats(0), o.stats(), f"after a call of {n}")
    assert_same_state(ctx.state(0), o.state(), "remainder graphs")
    ctx.close()
