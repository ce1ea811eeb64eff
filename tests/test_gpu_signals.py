"""Fixed-time signals on the GPU, in both step modes, against the oracle."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S
from parity import assert_same_state, assert_same_stats, run_side_by_side

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1])
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
