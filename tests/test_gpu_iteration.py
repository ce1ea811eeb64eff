"""The iteration series on the GPU: every run equals the oracle on the same
plans, the series is deterministic, and re-tiling from measured costs
changes nothing but the tiling."""
import pytest

import oracle
from paper_cs_0105004_amd import iteration as I
from paper_cs_0105004_amd import scenarios as S
from parity import assert_same_state

pytestmark = pytest.mark.gpu


def test_series_runs_match_oracle_and_repeat():
    scen = S.portland_like(scale=0.02, T=400)
    a = I.run_series(scen, n_runs=4, frac=0.2, seed=5, feedback=True)
    b = I.run_series(scen, n_runs=4, frac=0.2, seed=5, feedback=False)
    assert [r["hash"] for r in a] == [r["hash"] for r in b]
    # the plans really change between runs
    assert len({r["hash"] for r in a}) == 4
    for r in (a[0], a[3]):
        o = oracle.OracleSim(r["scenario"])
        o.step(r["scenario"].T)
        assert o.stats()["hash"] == r["hash"]
    # and the last run's full state
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=1)
    ctx.load(0, a[3]["scenario"])
    ctx.step(0, 400)
    o = oracle.OracleSim(a[3]["scenario"])
    o.step(400)
    assert_same_state(ctx.state(0), o.state(), "run 3")
    ctx.close()
