"""Side-by-side runs of the GPU library and the CPU oracle on one scenario."""
import numpy as np

import oracle

STAT_KEYS = ("t", "n_waiting", "n_active", "n_arrived", "veh_updates", "sum_v",
             "crossings", "exits", "lane_changes", "insertions", "c_occ",
             "hash")
STATE_KEYS = ("status", "link", "lane", "x", "v", "rptr", "exit_t")


def assert_same_state(g, o, where=""):
    for k in STATE_KEYS:
        if k not in o:
            continue
        a, b = np.asarray(g[k]), np.asarray(o[k])
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b)
            raise AssertionError(
                f"{where}: {k} differs at {len(bad)} entries, first ids "
                f"{bad[:8].tolist()} gpu={a[bad[:8]].tolist()} "
                f"oracle={b[bad[:8]].tolist()}")


def assert_same_stats(g, o, where=""):
    for k in STAT_KEYS:
        assert g[k] == o[k], f"{where}: stat {k}: gpu={g[k]} oracle={o[k]}"


def run_side_by_side(ctx, slot, scen, steps, every=1, full_at=()):
    """Steps both simulators; compares counters and the state hash every
    `every` steps and the whole state at the steps listed in full_at and at
    the end."""
    ctx.load(slot, scen)
    orc = oracle.OracleSim(scen)
    done = 0
    full_at = set(full_at) | {steps}
    while done < steps:
        k = min(every, steps - done)
        ctx.step(slot, k)
        orc.step(k)
        done += k
        assert_same_stats(ctx.stats(slot), orc.stats(), f"{scen.name} t={done}")
        if done in full_at:
            assert_same_state(ctx.state(slot), orc.state(),
                              f"{scen.name} t={done}")
    return orc
