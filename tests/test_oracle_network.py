"""Pins for the oracle's network update: parking, lane change, intersections
and the move across links (Section "Microsimulation driving logic";
readings R5-R8 in the oracle)."""
import numpy as np
import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S

from hand_cases import BOUNDARIES, build, check, load_cases


@pytest.mark.parametrize("case", load_cases() + load_cases(BOUNDARIES),
                         ids=lambda c: c["name"])
def test_hand_worked_cases(case):
    o = oracle.OracleSim(build(case))
    o.step(case["steps"])
    check(case, o.state(), o.stats())


def ring_of_loop(scen):
    """The periodic ring a single-lane loop of links unrolls to."""
    starts = np.concatenate([[0], np.cumsum(scen.link_len)[:-1]])
    cells = starts[scen.route_links[scen.route_off[:-1]]] + scen.init_x
    return S.ring_from_cells(int(scen.link_len.sum()), cells.astype(np.int32),
                             scen.init_v, scen.vmax, "0", scen.seed, scen.T)


@pytest.mark.parametrize("p", ["0", "0.2", "0.5"])
def test_loop_of_links_equals_ring(p):
    # a single lane loop of links is the ring of their total length: the lone
    # candidate at each node sees (len-1-x) + min(vmax, x_rear), which brakes
    # it exactly like the ring gap since v1 <= vmax
    rng = np.random.Generator(np.random.PCG64(21))
    for trial in range(12):
        k = int(rng.integers(2, 7))
        lengths = rng.integers(6, 40, size=k)
        total = int(lengths.sum())
        n = int(rng.integers(1, total // 2))
        loop = S.loop_of_links(lengths, n, vmax=5, p=p, seed=trial, T=150,
                               placement_seed=trial)
        ringsc = ring_of_loop(loop)
        ringsc.slow_thr = loop.slow_thr
        starts = np.concatenate([[0], np.cumsum(lengths)[:-1]])
        a, b = oracle.OracleSim(loop), oracle.OracleSim(ringsc)
        for t in range(150):
            a.step(1)
            b.step(1)
            sa, sb = a.state(), b.state()
            assert (sa["status"] == S.ACTIVE).all()
            assert np.array_equal(starts[sa["link"]] + sa["x"], sb["x"]), t
            assert np.array_equal(sa["v"], sb["v"]), t
        assert a.stats()["sum_v"] == b.stats()["sum_v"]


def test_two_lanes_without_lane_change_are_independent():
    lengths = [12, 20, 9, 15]
    both = S.loop_of_links(lengths, 10, vmax=5, p="0.3", seed=4, T=120,
                           lanes=2, placement_seed=3)
    n = 10

    def only(lane):
        s = S.loop_of_links(lengths, 10, vmax=5, p="0.3", seed=4, T=120,
                            lanes=2, placement_seed=3)
        drop = s.init_lane != lane
        s.init_status = np.where(drop, S.ARRIVED, S.ACTIVE).astype(np.int8)
        return s

    o = oracle.OracleSim(both)
    o0, o1 = oracle.OracleSim(only(0)), oracle.OracleSim(only(1))
    o.step(120)
    o0.step(120)
    o1.step(120)
    s, s0, s1 = o.state(), o0.state(), o1.state()
    for key in ("link", "lane", "x", "v", "rptr"):
        assert np.array_equal(s[key][:n], s0[key][:n])
        assert np.array_equal(s[key][n:], s1[key][n:])


def free_flow_exit_times(lengths, depart, vmax):
    """Closed form for a lone vehicle at p = 0: after k moves it has covered
    sum_{s=1..k} min(s, vmax) cells; it leaves link j in the step in which
    that distance first reaches the cumulative length of links 0..j."""
    ends = np.cumsum(lengths)
    out = []
    dist, k = 0, 0
    for e in ends:
        while dist < e:
            k += 1
            dist += min(k, vmax)
        out.append(depart + k - 1)
    return out


@pytest.mark.parametrize("vmax", [1, 3, 5, 7])
def test_lone_vehicle_free_flow_exit_times(vmax):
    rng = np.random.Generator(np.random.PCG64(vmax))
    for trial in range(10):
        k = int(rng.integers(1, 8))
        lengths = rng.integers(vmax + 1, 60, size=k)
        d = int(rng.integers(0, 20))
        scen = S.chain(lengths, depart=(d,), vmax=vmax, p="0", T=400)
        o = oracle.OracleSim(scen)
        o.step(d + int(lengths.sum()) + 5)
        st = o.state()
        assert st["status"][0] == S.ARRIVED
        assert st["exit_t"].tolist() == free_flow_exit_times(lengths, d, vmax)


@pytest.fixture(scope="module")
def small_grid():
    return S.portland_like(scale=0.01, T=400, depart_max=150)


def test_grid_lifecycle_and_priority_invariants(small_grid):
    scen = small_grid
    o = oracle.OracleSim(scen)
    N = scen.n_veh
    L = scen.n_links
    vmax = scen.vmax
    insert_t = np.full(N, -1)
    prev = o.state()
    origin = scen.route_links[scen.route_off[:-1]]
    for t in range(scen.T):
        o.step(1)
        st = o.state()
        stats = o.stats()
        assert stats["n_waiting"] + stats["n_active"] + stats["n_arrived"] == N
        newly = (prev["status"] == S.WAITING) & (st["status"] != S.WAITING)
        insert_t[newly] = t
        # at most one insertion per link per step
        assert np.bincount(origin[newly], minlength=L).max(initial=0) <= 1
        act = st["status"] == S.ACTIVE
        # no two vehicles in one cell
        key = (st["link"][act].astype(np.int64) * 8 + st["lane"][act]) * 40000 \
            + st["x"][act]
        assert len(np.unique(key)) == act.sum()
        assert ((st["v"] >= 0) & (st["v"] <= vmax)).all()
        # crossings: vehicles active before and after whose rptr advanced
        was = prev["status"] == S.ACTIVE
        crossed = np.flatnonzero(was & act & (st["rptr"] > prev["rptr"]))
        tgt = st["link"][crossed].astype(np.int64) * 8 + st["lane"][crossed]
        assert len(np.unique(tgt)) == len(crossed)  # one per target lane
        # priority: no candidate of smaller (rank, lane) aimed at that lane
        cand = np.flatnonzero(was)
        lead = {}
        for i in cand:
            q = (prev["link"][i], prev["lane"][i])
            if q not in lead or prev["x"][i] > prev["x"][lead[q]]:
                lead[q] = i
        aims = {}
        for (l, k), i in lead.items():
            if scen.link_len[l] - 1 - prev["x"][i] >= vmax:
                continue
            r = scen.route_off[i] + prev["rptr"][i]
            if r + 1 >= scen.route_off[i + 1]:
                continue
            nl = scen.route_links[r + 1]
            nk = min(k, scen.link_lanes[nl] - 1)
            aims.setdefault((nl, nk), []).append((scen.link_rank[l], k, i))
        for i in crossed:
            tl = (st["link"][i], st["lane"][i])
            best = min(aims[tl])
            assert best[2] == i
        prev = st
    st = o.state()
    # insertion never precedes the departure time; FIFO per origin link
    ins = insert_t >= 0
    assert (insert_t[ins] >= scen.depart[ins]).all()
    for l in range(L):
        ids = np.flatnonzero(ins & (origin == l))
        order = np.lexsort((ids, scen.depart[ids]))
        assert (np.diff(insert_t[ids[order]]) > 0).all()
    # exit times strictly increase along every route
    for i in range(N):
        e = st["exit_t"][scen.route_off[i]:scen.route_off[i + 1]]
        done = e[e >= 0]
        assert (np.diff(done) > 0).all()
        assert (e[:len(done)] >= 0).all()


def test_no_incentive_no_lane_change():
    # vehicles spaced more than vmax apart in every lane never want to change
    lengths = [40, 55, 47]
    base = S.loop_of_links(lengths, 1, vmax=5, p="0", seed=2, T=100, lanes=3,
                           placement_seed=5)
    lc = S.loop_of_links(lengths, 1, vmax=5, p="0", seed=2, T=100, lanes=3,
                         placement_seed=5, flags=S.FLAG_LANE_CHANGE)
    a, b = oracle.OracleSim(base), oracle.OracleSim(lc)
    a.step(100)
    b.step(100)
    assert b.stats()["lane_changes"] == 0
    for key in ("link", "lane", "x", "v"):
        assert np.array_equal(a.state()[key], b.state()[key])


def test_single_lane_links_ignore_lane_change():
    lengths = [12, 20, 9, 15]
    a = S.loop_of_links(lengths, 20, vmax=5, p="0.2", seed=4, T=100)
    b = S.loop_of_links(lengths, 20, vmax=5, p="0.2", seed=4, T=100,
                        flags=S.FLAG_LANE_CHANGE)
    oa, ob = oracle.OracleSim(a), oracle.OracleSim(b)
    oa.step(100)
    ob.step(100)
    assert oa.stats()["hash"] == ob.stats()["hash"]


def test_lane_change_conserves_and_changes(small_grid):
    import dataclasses
    scen = dataclasses.replace(small_grid,
                               flags=S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES)
    scen.conn_off, scen.conn_out, scen.conn_lo, scen.conn_hi = \
        S._ranks_and_conn(scen.n_nodes, scen.link_from, scen.link_to,
                          scen.link_lanes, scen.node_xy, True)[1:]
    o = oracle.OracleSim(scen)
    o.step(300)  # raises if two vehicles ever share a cell
    st = o.stats()
    assert st["lane_changes"] > 0
    assert st["n_waiting"] + st["n_active"] + st["n_arrived"] == scen.n_veh


def test_restart_from_saved_state(small_grid):
    scen = small_grid
    a = oracle.OracleSim(scen)
    a.step(150)
    mid = a.state()
    a.step(100)
    b = oracle.OracleSim(scen.with_state(mid, 150))
    b.step(100)
    sa, sb = a.state(), b.state()
    for key in sa:
        assert np.array_equal(sa[key], sb[key]), key


def test_lane_change_draw_is_sub_step_0():
    # reading R3: a vehicle that qualifies for a discretionary change takes
    # it iff word 0 of Philox4x32-10 at counter (id, t, 0, 0) is below
    # lc_thr (the Philox function itself is pinned to rocRAND's)
    import dataclasses
    case = next(c for c in load_cases() if c["name"] == "lc_discretionary_one_side")
    base = build(case)
    taken = []
    for seed in range(1, 65):
        scen = dataclasses.replace(base, seed=seed, lc_thr=1 << 31)
        o = oracle.OracleSim(scen)
        o.step(1)
        lane = int(o.state()["lane"][0])
        o.close()
        u = int(oracle.philox4x32_10(np.array([0, 0, 0, 0], np.uint32),
                                     np.array([seed, 0], np.uint32))[0])
        assert lane == (1 if u < (1 << 31) else 0), seed
        taken.append(lane)
    assert 0 < sum(taken) < len(taken)  # both outcomes occur
