"""Pins of the oracle's fixed-time signals (readings S1-S3): a light that is
never red changes nothing, a light that is never green lets nobody through,
a lone vehicle's exit time has a closed form, and on a signalised grid no
vehicle ever leaves a link while its light is red."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S


def with_plan(scen, plan_of_link, cycle, red, offset):
    """The scenario with one signal plan on the given links."""
    plan = np.full(scen.n_links, -1, np.int8)
    plan[plan_of_link] = 0
    return dataclasses.replace(
        scen, signal_plan=plan, plan_cycle=np.array([cycle], np.int32),
        plan_red=np.array([red], np.int32),
        plan_offset=np.array([offset], np.int32))


def run(scen, steps):
    o = oracle.OracleSim(scen)
    o.step(steps)
    return o.stats(), o.state()


def test_never_red_changes_nothing():
    base = S.portland_like(scale=0.02, T=300)
    green = with_plan(base, np.arange(base.n_links), cycle=17, red=0, offset=3)
    a, sa = run(base, 300)
    b, sb = run(green, 300)
    assert a == b
    for k in sa:
        np.testing.assert_array_equal(sa[k], sb[k])


def test_never_green_holds_everyone_on_the_first_link():
    scen = S.chain([40, 40], depart=(0, 3, 6, 9, 12), p="0.2", T=200)
    red = with_plan(scen, [0], cycle=10, red=10, offset=0)
    st, state = run(red, 200)
    assert st["crossings"] == 0 and st["exits"] == 0
    assert (state["exit_t"] == -1).all()
    assert (state["rptr"][state["status"] == 1] == 0).all()
    # they queue up against the virtual vehicle, the first at the last cell
    assert state["x"].max() == 39


def free_flow_crossing_step(length, vmax):
    """The step in which a lone vehicle entering at cell 0 with speed 0 in
    step 0 first reaches cell `length` (positions 1, 3, 6, ... capped)."""
    x, s = 0, 0
    while True:
        x += min(s + 1, vmax)
        if x >= length:
            return s
        s += 1


@pytest.mark.parametrize("cycle,red,offset", [(20, 10, 0), (20, 10, 7),
                                              (30, 25, 3), (9, 1, 4),
                                              (60, 30, 30)])
@pytest.mark.parametrize("vmax", [1, 3, 5])
def test_lone_vehicle_waits_for_green(cycle, red, offset, vmax):
    # p = 0: the vehicle crosses in its free-flow step if that step is green,
    # else in the first green step after it (it waits at the last cell)
    length = 37
    scen = S.chain([length, 25], depart=(0,), vmax=vmax, p="0", T=300)
    sig = with_plan(scen, [0], cycle, red, offset)
    _, state = run(sig, 300)
    t_free = free_flow_crossing_step(length, vmax)
    is_red = lambda t: (t + offset) % cycle < red
    t_exp = t_free
    while is_red(t_exp):
        t_exp += 1
    assert state["exit_t"][0] == t_exp


def test_no_crossing_on_red_in_a_signalised_grid():
    scen = S.portland_like(scale=0.03, T=500, signals=(40, 20))
    st, state = run(scen, 500)
    assert st["crossings"] > 0
    plan = scen.signal_plan[scen.route_links]
    off = scen.plan_offset[np.maximum(plan, 0)]
    left = state["exit_t"] >= 0
    red = (plan >= 0) & ((state["exit_t"] + off) % 40 < 20)
    assert not (left & red).any()
    # the unsignalised run moves more vehicles through the same network
    plain = dataclasses.replace(scen, signal_plan=None, plan_cycle=None,
                                plan_red=None, plan_offset=None)
    st0, _ = run(plain, 500)
    assert st0["exits"] > st["exits"]


def test_plan_validation():
    scen = S.chain([40, 40], depart=(0,), T=10)
    for cycle, red, offset in [(0, 0, 0), (10, 11, 0), (10, -1, 0),
                               (10, 5, -1)]:
        with pytest.raises(oracle.OracleError):
            oracle.OracleSim(with_plan(scen, [0], cycle, red, offset))
