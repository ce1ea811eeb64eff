"""Builds Scenario inputs from the hand-worked cases in golden/hand_cases.json
and checks a simulator's end state against the recorded outcome."""
import json
import os

import numpy as np

from paper_cs_0105004_amd import scenarios as S

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PATH = os.path.join(GOLDEN, "hand_cases.json")
BOUNDARIES = os.path.join(GOLDEN, "hand_cases_boundaries.json")
FLAGS = {"LANE_CHANGE": S.FLAG_LANE_CHANGE, "TURN_LANES": S.FLAG_TURN_LANES}
STATUS = {"waiting": S.WAITING, "active": S.ACTIVE, "arrived": S.ARRIVED}


def load_cases(path=PATH):
    with open(path) as f:
        return json.load(f)["cases"]


def build(case) -> S.Scenario:
    links = np.array(case["links"], np.int64).reshape(-1, 5)
    L = len(links)
    conn = sorted(case.get("conn", []))
    conn_off = np.zeros(L + 1, np.int64)
    for c in conn:
        conn_off[c[0] + 1] += 1
    conn_off = np.cumsum(conn_off)
    vehs = case["vehicles"]
    n = len(vehs)
    route_off = np.zeros(n + 1, np.int64)
    np.cumsum([len(v["route"]) for v in vehs], out=route_off[1:])
    status = np.array([S.WAITING if "depart" in v else S.ACTIVE for v in vehs],
                      np.int8)
    flags = 0
    for f in case.get("flags", []):
        flags |= FLAGS[f]
    nn = case["nodes"]
    return S.Scenario(
        name=case["name"], flags=flags, vmax=case["vmax"],
        slow_thr=S.prob_threshold(case.get("p", "0")),
        seed=case.get("seed", 1), T=case["steps"], n_nodes=nn,
        link_from=links[:, 0].astype(np.int32),
        link_to=links[:, 1].astype(np.int32),
        link_len=links[:, 2].astype(np.int32),
        link_lanes=links[:, 3].astype(np.int8),
        link_rank=links[:, 4].astype(np.int8),
        conn_off=conn_off,
        conn_out=np.array([c[1] for c in conn], np.int32),
        conn_lo=np.array([c[2] for c in conn], np.int8),
        conn_hi=np.array([c[3] for c in conn], np.int8),
        node_xy=np.stack([np.arange(nn), np.zeros(nn)], 1).astype(float),
        n_veh=n,
        depart=np.array([v.get("depart", 0) for v in vehs], np.int32),
        route_off=route_off,
        route_links=np.concatenate([v["route"] for v in vehs]).astype(np.int32),
        init_status=status,
        init_lane=np.array([v.get("lane", 0) for v in vehs], np.int8),
        init_x=np.array([v.get("x", 0) for v in vehs], np.int32),
        init_v=np.array([v.get("v", 0) for v in vehs], np.int8),
        init_rptr=np.zeros(n, np.int32))


def check(case, state, stats):
    """Assert a simulator's state/stats after case['steps'] steps match."""
    for i, e in enumerate(case["expect"]):
        st = STATUS[e.get("status", "active")]
        assert state["status"][i] == st, (case["name"], i, "status")
        if st != S.ACTIVE:
            continue
        for key in ("link", "lane", "x", "v", "rptr"):
            if key in e:
                assert int(state[key][i]) == e[key], (case["name"], i, key)
    if "exit_t" in case:
        ro = np.cumsum([0] + [len(v["route"]) for v in case["vehicles"]])
        for i, row in enumerate(case["exit_t"]):
            got = state["exit_t"][ro[i]:ro[i + 1]].tolist()
            assert got == row, (case["name"], i, "exit_t")
    for key, val in case.get("stats", {}).items():
        assert stats[key] == val, (case["name"], key)
