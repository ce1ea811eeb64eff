"""The 200,000-link network with lane changing and turn lanes: exact
parity with the oracle on a scaled-down copy over its whole horizon; at
full size on the first steps (all 2M vehicles' state), over the whole
7,200-step horizon against the oracle's checkpoints at t = 1,800, 3,600 and
7,200, and properties that hold at any size."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S
from parity import assert_same_state, assert_same_stats, run_side_by_side

pytestmark = pytest.mark.gpu


def test_large_network_scaled_down_matches_oracle():
    from paper_cs_0105004_amd.sim import Context
    scen = S.large_network(scale=0.005, T=1500)
    assert scen.flags & S.FLAG_LANE_CHANGE and scen.flags & S.FLAG_TURN_LANES
    ctx = Context(max_slots=1)
    o = run_side_by_side(ctx, 0, scen, 1500, every=250, full_at=(500, 1000))
    st = o.stats()
    assert st["lane_changes"] > 0 and st["exits"] > 0
    ctx.close()


@pytest.fixture(scope="module")
def full():
    return S.large_network()


def test_large_network_full_size_first_steps_match_oracle(full):
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=1)
    ctx.load(0, full)
    ctx.step(0, 300)
    o = oracle.OracleSim(full)
    o.step(300)
    assert_same_stats(ctx.stats(0), o.stats(), "full size t=300")
    assert_same_state(ctx.state(0), o.state(), "full size t=300")
    assert o.stats()["n_active"] + o.stats()["n_arrived"] > 20000
    ctx.close()


def test_large_network_full_horizon_properties(full):
    from paper_cs_0105004_amd.sim import Context
    n = full.n_veh
    a = Context(max_slots=1)  # the default launch configuration
    a.load(0, full)
    for t in range(0, full.T, 1800):
        a.step(0, 1800)
        st = a.stats(0)
        assert st["n_waiting"] + st["n_active"] + st["n_arrived"] == n
        assert st["dev_err"] == 0
    end = a.state(0)
    # exit times along each route increase strictly where set (sample)
    rng = np.random.Generator(np.random.PCG64(3))
    for i in rng.choice(n, size=2000, replace=False):
        e = end["exit_t"][full.route_off[i]:full.route_off[i + 1]]
        e = e[e >= 0]
        assert np.all(np.diff(e) > 0), i
        assert np.all(e >= full.depart[i])
    # another tiling and launch shape gives the same final state
    b = Context(max_slots=1, tile_lanes=64, back_pieces=1, graph_steps=-1)
    b.load(0, full)
    b.step(0, full.T)
    assert b.stats(0)["hash"] == a.stats(0)["hash"]
    assert_same_state(b.state(0), end, "tilings")
    a.close()
    b.close()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "large_network_checkpoints.json")
STATE_DTYPES = (("status", np.int8), ("link", np.int32), ("lane", np.int8),
                ("x", np.int32), ("v", np.int8), ("rptr", np.int32),
                ("exit_t", np.int32))


def _digests(state):
    out = {}
    for key, dt in STATE_DTYPES:
        a = np.ascontiguousarray(state[key],
                                 dtype=np.dtype(dt).newbyteorder("<"))
        out[key] = hashlib.sha256(a.tobytes()).hexdigest()
    return out


def test_large_network_full_horizon_matches_oracle_checkpoints(full):
    """All 2,000,000 vehicles over the whole 7,200 steps in the default
    launch configuration, against the checkpoints that
    golden/make_large_network_checkpoints.py wrote from the oracle alone:
    every counter, the state hash, and SHA-256 digests of every per-vehicle
    state array and of the exit-time array."""
    from paper_cs_0105004_amd.sim import Context
    with open(GOLDEN) as f:
        cps = {c["stats"]["t"]: c for c in json.load(f)["checkpoints"]}
    assert sorted(cps) == [1800, 3600, 7200]
    ctx = Context(max_slots=1)
    ctx.load(0, full)
    t = 0
    for cp in sorted(cps):
        ctx.step(0, cp - t)
        t = cp
        got = ctx.stats(0)
        print("checkpoint", cp, "active", got["n_active"], flush=True)
        for k, v in cps[cp]["stats"].items():
            assert got[k] == v, f"t={cp} {k}: gpu={got[k]} oracle={v}"
        assert got["dev_err"] == 0
        d = _digests(ctx.state(0))
        for k, v in cps[cp]["sha256"].items():
            assert d[k] == v, f"t={cp}: {k} differs from the oracle's"
    ctx.close()
