"""Pins for the oracle's state hash (reading R10: a sum over vehicles, mod
2^64, of a mix of each vehicle's id, status and, when active, link, lane,
cell, speed and route pointer).

The GPU parity tests compare the whole state as well as the hash, but
several checks (the bench's oracle check, restarts, served runs) compare
the hash alone, so it must see every field.  Two properties pin it without
restating its formula: changing any single field of one vehicle changes
the hash, and the change a vehicle makes does not depend on the other
vehicles (the hash is a sum over vehicles)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S


@pytest.fixture(scope="module")
def loop():
    # two lanes around a cycle of three links; every route repeats the cycle
    return S.loop_of_links([40, 50, 60], 10, vmax=5, p="0", seed=3, T=50,
                           lanes=2, placement_seed=4)


def state_hash(scen):
    o = oracle.OracleSim(scen)
    h = o.stats()["hash"]
    o.close()
    return h


def changed(scen, i, **fields):
    s = dataclasses.replace(scen)
    for name, val in fields.items():
        if name == "route_shift":  # the same route, started one link later
            rl = s.route_links.copy()
            a, b = s.route_off[i], s.route_off[i + 1]
            rl[a:b] = (rl[a:b] + val) % s.n_links
            s.route_links = rl
            continue
        arr = getattr(s, name).copy()
        arr[i] = val
        setattr(s, name, arr)
    return s


def free_vehicle(scen):
    """An active vehicle whose next cell and the cell beside it are empty,
    and whose link's successor has its cell x empty in its lane too."""
    link = scen.route_links[scen.route_off[:-1] + scen.init_rptr]
    occ = {(int(l), int(k), int(x)) for l, k, x in
           zip(link, scen.init_lane, scen.init_x)}
    for i in range(scen.n_veh):
        l, k, x = int(link[i]), int(scen.init_lane[i]), int(scen.init_x[i])
        nxt = (l + 1) % scen.n_links
        if (x + 1 < scen.link_len[l] and (l, k, x + 1) not in occ
                and (l, 1 - k, x) not in occ and (nxt, k, x) not in occ
                and x < scen.link_len[nxt]):
            return i
    raise AssertionError("no free vehicle")


def test_every_field_moves_the_hash(loop):
    i = free_vehicle(loop)
    base = state_hash(loop)
    k = loop.n_links
    variants = {
        "cell": dict(init_x=loop.init_x[i] + 1),
        "speed": dict(init_v=loop.init_v[i] + 1),
        "lane": dict(init_lane=1 - loop.init_lane[i]),
        "route pointer (same link, one lap on)": dict(init_rptr=loop.init_rptr[i] + k),
        "link (same pointer, route shifted)": dict(route_shift=1),
        "status": dict(init_status=S.ARRIVED),
    }
    seen = {base}
    for name, f in variants.items():
        h = state_hash(changed(loop, i, **f))
        assert h != base, name
        seen.add(h)
    assert len(seen) == len(variants) + 1  # all different from each other too


def test_hash_is_a_sum_over_vehicles(loop):
    i = free_vehicle(loop)
    j = (i + 3) % loop.n_veh
    mod = 1 << 64
    for f in (dict(init_x=loop.init_x[i] + 1), dict(init_status=S.ARRIVED)):
        for other in (loop, changed(loop, j, init_v=2)):
            d = (state_hash(changed(other, i, **f)) - state_hash(other)) % mod
            if other is loop:
                first = d
            else:
                assert d == first  # vehicle i's part does not see vehicle j
