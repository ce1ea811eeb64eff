"""Full-size parity on the Portland-sized network (20,024 links, 200,000
vehicles, 3,600 steps) in the configuration the benchmark times: the GPU run
and the CPU oracle must end in the same state, vehicle by vehicle, with the
same exit times and counters."""
import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S

from parity import assert_same_state, assert_same_stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def portland():
    return S.portland_like()


def test_portland_full_run_matches_oracle(portland):
    from paper_cs_0105004_amd.sim import Context
    ctx = Context(max_slots=1)  # the benchmark's default launch configuration
    ctx.load(0, portland)
    orc = oracle.OracleSim(portland)
    for upto in (900, 1800, 3600):
        ctx.step(0, upto - ctx.stats(0)["t"])
        orc.step(upto - orc.stats()["t"])
        print("portland step", upto, flush=True)
        assert_same_stats(ctx.stats(0), orc.stats(), f"portland t={upto}")
    assert_same_state(ctx.state(0), orc.state(), "portland end")
    ctx.close()


# Launch configurations that change the number of workgroups by 40x: with
# tiles of one lane, many more workgroups run than fit on the device at once,
# so a tile may run long after the tiles it reads from -- every read of
# another tile's data must see the previous step's values regardless.
@pytest.mark.parametrize("mode,lanes,cells,pieces,graph", [
    (1, 16, 0, 1, -1), (1, 16, 0, 8, 200), (1, 1, 0, 1, 64),
    (0, 1, 0, 1, 64), (0, 4, 256, 1, 32), (0, 64, 65536, 1, 64),
    (2, 16, 0, 1, 64), (2, 1, 0, 1, 64)])
def test_portland_configs_agree(portland, mode, lanes, cells, pieces, graph):
    from paper_cs_0105004_amd.sim import Context
    ref = Context(max_slots=1)
    alt = Context(max_slots=1, step_mode=mode, tile_lanes=lanes,
                  tile_cells=cells, back_pieces=pieces, graph_steps=graph)
    ref.load(0, portland)
    alt.load(0, portland)
    ref.step(0, 1500)
    alt.step(0, 1500)
    assert_same_stats(alt.stats(0), ref.stats(0), "configs")
    assert_same_state(alt.state(0), ref.state(0), "configs")
    ref.close()
    alt.close()


def test_batched_replications_full_size_sampled():
    # all 64 replications (417k links, 4.1M vehicles) in the launch
    # configuration the batched benchmark picks, full 3,600 steps; the three
    # smallest are compared with the oracle vehicle by vehicle, every one
    # against counters that hold at any size
    import numpy as np
    from paper_cs_0105004_amd.sim import Context
    scens = S.batched_scenarios()
    ctx = Context(max_slots=len(scens), tile_lanes=64, tile_cells=16384,
                  graph_steps=64)
    for k, sc in enumerate(scens):
        ctx.load(k, sc)
    ctx.step(list(range(len(scens))), 3600)
    for k, sc in enumerate(scens):
        st = ctx.stats(k)
        assert st["dev_err"] == 0
        assert st["n_waiting"] + st["n_active"] + st["n_arrived"] == sc.n_veh
        assert st["insertions"] == sc.n_veh - st["n_waiting"]
        assert st["exits"] == st["n_arrived"]
    order = np.argsort([sc.n_veh for sc in scens])[:3]
    for k in order:
        o = oracle.OracleSim(scens[k])
        o.step(3600)
        print("replication", k, scens[k].n_links, "links", flush=True)
        assert_same_stats(ctx.stats(k), o.stats(), f"replication {k}")
        assert_same_state(ctx.state(k), o.state(), f"replication {k}")
    ctx.close()
