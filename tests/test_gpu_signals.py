"""Fixed-time signals on the GPU, in both step modes, against the oracle."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S
from parity import assert_same_state, assert_same_stats, run_side_by_side

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("cycle,red", [(40, 20), (60, 30), (7, 3)])
def test_signalised_grid(mode, cycle, red):
    from paper_cs_0105004_amd.sim import Context
    scen = S.portland_like(scale=0.03, T=500, signals=(cycle, red))
    ctx = Context(max_slots=1, step_mode=mode)
    run_side_by_side(ctx, 0, scen, 500, every=50, full_at=(100, 250))
    ctx.close()


@pytest.mark.parametrize("flags", [S.FLAG_LANE_CHANGE,
                                   S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES])
def test_signalised_grid_with_lane_changes(flags):
    from paper_cs_0105004_amd.sim import Context
    scen = S.portland_like(scale=0.03, T=400, flags=flags, signals=(30, 15))
    ctx = Context(max_slots=1)
    o = run_side_by_side(ctx, 0, scen, 400, every=40, full_at=(200,))
    assert o.stats()["lane_changes"] > 0
    ctx.close()


def test_signalised_and_plain_slots_in_one_launch():
    from paper_cs_0105004_amd.sim import Context
    scens = [S.portland_like(scale=0.02, T=300, signals=(40, 20)),
             S.portland_like(scale=0.02, T=300, seed=7),
             S.portland_like(scale=0.02, T=300, seed=8, signals=(10, 9))]
    ctx = Context(max_slots=3)
    for k, sc in enumerate(scens):
        ctx.load(k, sc)
    ctx.step([0, 1, 2], 300)
    for k, sc in enumerate(scens):
        o = oracle.OracleSim(sc)
        o.step(300)
        assert_same_stats(ctx.stats(k), o.stats(), f"slot {k}")
        assert_same_state(ctx.state(k), o.state(), f"slot {k}")
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_lone_vehicles_at_a_light(mode):
    from paper_cs_0105004_amd.sim import Context
    scen = S.chain([37, 25, 40], depart=(0, 5, 11, 30), vmax=5, p="0.3",
                   T=250)
    plan = np.array([0, 1, -1], np.int8)
    scen = dataclasses.replace(
        scen, signal_plan=plan, plan_cycle=np.array([20, 9], np.int32),
        plan_red=np.array([10, 8], np.int32),
        plan_offset=np.array([7, 0], np.int32))
    ctx = Context(max_slots=1, step_mode=mode)
    run_side_by_side(ctx, 0, scen, 250, every=1, full_at=(50, 100))
    ctx.close()


def _red(scen, link, t):
    j = int(scen.signal_plan[link])
    if j < 0:
        return False
    c, r, o = (int(scen.plan_cycle[j]), int(scen.plan_red[j]),
               int(scen.plan_offset[j]))
    return (t + o) % c < r


def _red_lead_beats_green(scen, st, t):
    """Is there a target lane that a lead vehicle held by a red light would
    claim with a smaller (rank, lane) key than a green candidate's?"""
    lead = {}
    for i in np.flatnonzero(st["status"] == S.ACTIVE):
        q = (int(st["link"][i]), int(st["lane"][i]))
        if q not in lead or st["x"][i] > st["x"][lead[q]]:
            lead[q] = i
    best = {}
    for (lk, k), i in lead.items():
        ro = scen.route_off[i]
        if (st["rptr"][i] + 1 == scen.route_off[i + 1] - ro
                or scen.link_len[lk] - 1 - st["x"][i] >= scen.vmax):
            continue
        nl = int(scen.route_links[ro + st["rptr"][i] + 1])
        tgt = (nl, min(k, int(scen.link_lanes[nl]) - 1))
        key = int(scen.link_rank[lk]) * 8 + k
        red, green = best.get(tgt, (1 << 30, -1))
        if _red(scen, lk, t):
            red = min(red, key)
        else:
            green = max(green, key)
        best[tgt] = (red, green)
    return any(red < green for red, green in best.values())


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_restart_at_a_red_phase(mode):
    """A restart from a saved state while lights are red: a lead vehicle at
    a red light claims nothing in the restart step, so a green candidate of
    lower priority for the same target lane still wins it.  (The one-kernel
    step registers the claims of the restart step on the host.)  The restart
    step is the first after step 300 at which such a pair exists."""
    from paper_cs_0105004_amd.sim import Context
    scen = S.portland_like(scale=0.03, T=800, signals=(40, 20))
    o = oracle.OracleSim(scen)
    o.step(300)
    t0 = 300
    while not _red_lead_beats_green(scen, o.state(), t0):
        assert t0 < 700, "no restart step with a red lead ahead of a green one"
        o.step(1)
        t0 += 1
    rs = scen.with_state(o.state(), t0)
    ctx = Context(max_slots=1, step_mode=mode)
    ctx.load(0, rs)
    for k in range(4):
        ctx.step(0, 1 if k < 3 else 100)
        o.step(1 if k < 3 else 100)
        # the counters restart at the saved step; state and hash must agree
        assert ctx.stats(0)["hash"] == o.stats()["hash"], (t0, k)
    assert_same_state(ctx.state(0), o.state(), f"restart t0={t0} mode {mode}")
    ctx.close()
