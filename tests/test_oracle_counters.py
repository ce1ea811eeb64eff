"""Pins for the oracle's step counters, which the benchmark's algorithmic
bytes are made of: each step's increments are recomputed from their
definitions out of the state before and after the step, on a grid run of
150 steps.

* insertions: vehicles that were waiting and are no longer;
* exits: vehicles that were active and have arrived;
* vehicle-updates: vehicles active in the move, i.e. active before the step
  plus those inserted;
* crossings: active vehicles whose route pointer advanced (by exactly one);
* C_occ (no lane changes): the cells of the lanes holding a vehicle in the
  move, i.e. the lanes of the vehicles active before and of those inserted;
* sum of speeds: the speeds after the step, plus, for each vehicle that
  exited, a speed between min(v+1, vmax) - 1 and min(v+1, vmax);
* lane changes (with lane changes on): at least the vehicles seen in
  another lane of the same link (for a vehicle that entered, another lane
  than the lowest one free at cell 0), at most that plus the crossings."""
import numpy as np
import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S

KEYS = ("insertions", "exits", "veh_updates", "crossings", "c_occ", "sum_v",
        "lane_changes")


def walk(scen, steps):
    o = oracle.OracleSim(scen)
    before, sb = o.state(), o.stats()
    for _ in range(steps):
        o.step(1)
        after, sa = o.state(), o.stats()
        yield before, after, {k: sa[k] - sb[k] for k in KEYS}
        before, sb = after, sa
    o.close()


@pytest.mark.parametrize("lane_change", [False, True])
def test_step_counters_from_their_definitions(lane_change):
    flags = (S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES) if lane_change else 0
    scen = S.portland_like(scale=0.02, T=150, depart_max=60, seed=23,
                           flags=flags)
    vmax, seen = scen.vmax, {k: 0 for k in KEYS}
    for b, a, d in walk(scen, 150):
        act_b = b["status"] == S.ACTIVE
        act_a = a["status"] == S.ACTIVE
        ins = (b["status"] == S.WAITING) & (a["status"] != S.WAITING)
        ext = act_b & (a["status"] == S.ARRIVED)
        assert (a["status"][ins] == S.ACTIVE).all()  # no exit on entry
        assert d["insertions"] == ins.sum()
        assert d["exits"] == ext.sum()
        assert d["veh_updates"] == act_b.sum() + ins.sum()
        stay = act_b & act_a
        adv = a["rptr"][stay] - b["rptr"][stay]
        assert set(np.unique(adv)) <= {0, 1}
        assert d["crossings"] == (adv == 1).sum()
        moved = (act_b | ins) & ~ext
        v1 = np.minimum(b["v"][ext].astype(int) + 1, vmax)
        base = int(a["v"][moved].astype(int).sum())
        assert base + (v1 - 1).clip(0).sum() <= d["sum_v"] <= base + v1.sum()
        if not lane_change:
            lanes = set(zip(b["link"][act_b], b["lane"][act_b])) | \
                set(zip(a["link"][ins], a["lane"][ins]))
            assert d["c_occ"] == sum(int(scen.link_len[l]) for l, _ in lanes)
        else:
            same = np.flatnonzero(stay)[adv == 0]  # still on the same link
            side = int((a["lane"][same] != b["lane"][same]).sum())
            # a vehicle that entered took the lowest lane whose cell 0 was
            # empty before the step, and may have changed lanes at once
            at0 = set(zip(b["link"][act_b & (b["x"] == 0)],
                          b["lane"][act_b & (b["x"] == 0)]))
            for i in np.flatnonzero(ins):
                l = int(a["link"][i])
                k0 = min(k for k in range(scen.link_lanes[l]) if (l, k) not in at0)
                side += int(a["lane"][i] != k0)
            assert side <= d["lane_changes"] <= side + d["crossings"]
        for k in KEYS:
            seen[k] += d[k]
    # the run exercised every counter
    assert all(seen[k] > 0 for k in KEYS if k != "lane_changes" or lane_change)
