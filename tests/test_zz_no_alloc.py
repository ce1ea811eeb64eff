"""sim_step_noalloc (the step entry point that allocates nothing) against
sim_step, through the C ABI: the same slots loaded from the same inputs in
two contexts, one stepped by each entry point, must end bit for bit alike.
Two calls in a row, the second on a smaller input, so that the second call
finds the first call's work list in the shared device scratch."""
import numpy as np
import pytest

from paper_cs_0105004_amd import scenarios as S
from parity import assert_same_state, assert_same_stats

pytestmark = pytest.mark.gpu


def _pair(scens, steps, mode=0):
    from paper_cs_0105004_amd.sim import Context
    a = Context(max_slots=len(scens), step_mode=mode)
    b = Context(max_slots=len(scens), step_mode=mode)
    slots = list(range(len(scens)))
    for k, sc in enumerate(scens):
        a.load(k, sc)
        b.load(k, sc)
    a.step(slots, steps)
    b.step_noalloc(slots, steps)
    for k, sc in enumerate(scens):
        ga, gb = a.stats(k), b.stats(k)
        assert_same_stats(gb, ga, f"{sc.name} slot {k}")
        assert_same_state(b.state(k), a.state(k), f"{sc.name} slot {k}")
    a.close()
    b.close()


def test_noalloc_equals_step_twice_second_smaller():
    big = [S.portland_like(scale=0.05, T=300, depart_max=200, seed=3),
           S.portland_like(scale=0.02, T=300, depart_max=200, seed=4,
                           flags=S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES),
           S.ring(1000, 150, 5, "0.2", seed=42)]
    print("call 1: three slots, 300 steps", flush=True)
    _pair(big, 300)
    small = [S.portland_like(scale=0.01, T=120, depart_max=60, seed=5)]
    print("call 2: one smaller slot, 120 steps", flush=True)
    _pair(small, 120)


def test_noalloc_repeated_calls_and_mixed_use():
    """Many short calls, interleaved with sim_step on the same context,
    equal one long sim_step run; the two-kernel form included."""
    from paper_cs_0105004_amd.sim import Context
    sc = S.portland_like(scale=0.03, T=400, depart_max=300, seed=9)
    ref = Context(max_slots=1, step_mode=1)
    ref.load(0, sc)
    ref.step(0, 400)
    c = Context(max_slots=1, step_mode=1)
    c.load(0, sc)
    done = 0
    for n in (1, 7, 64, 3, 100, 25, 200):
        if done % 2:
            c.step(0, n)
        else:
            c.step_noalloc(0, n)
        done += n
    assert done == 400
    assert_same_stats(c.stats(0), ref.stats(0), "mixed calls")
    assert_same_state(c.state(0), ref.state(0), "mixed calls")
    c.close()
    ref.close()


def test_noalloc_rejects_bad_calls_without_stepping():
    from paper_cs_0105004_amd.sim import Context, SimError
    sc = S.portland_like(scale=0.01, T=50, depart_max=20, seed=2)
    c = Context(max_slots=2)
    c.load(0, sc)
    t = c.stats(0)["t"]
    with pytest.raises(SimError):
        c.step_noalloc([0, 0], 5)  # a slot listed twice
    with pytest.raises(SimError):
        c.step_noalloc([1], 5)  # not loaded
    assert c.stats(0)["t"] == t
    c.step_noalloc(0, 0)
    assert c.stats(0)["t"] == t
    c.close()
    np.testing.assert_equal(t, 0)
