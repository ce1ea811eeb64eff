"""CPU-side checks of the library's input validation through the C ABI.

sim_footprint takes no context and touches no device, and it runs the same
network and route-offset checks that sim_load_network and sim_load_vehicles
run before any device work: malformed input is refused with SIM_E_INVAL
instead of being read or written out of bounds."""
import ctypes as C
import dataclasses
import os

import numpy as np
import pytest

from paper_cs_0105004_amd import scenarios as S
from paper_cs_0105004_amd import sim


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sim.LIB_PATH):
        from paper_cs_0105004_amd import build
        build.build()
    return sim.load_library()


@pytest.fixture(scope="module")
def scen():
    return S.portland_like(scale=0.02, T=200, seed=9)


def footprint(lib, scen, link_cost=None, with_vehicles=True):
    inp = sim._Inputs(scen, link_cost)
    b = C.c_uint64(0)
    rc = lib.sim_footprint(None, C.byref(inp.params), C.byref(inp.net),
                           C.byref(inp.veh) if with_vehicles else None,
                           C.byref(b))
    return rc, int(b.value)


def with_routes(scen, route_off):
    return dataclasses.replace(scen, route_off=np.asarray(route_off, np.int64))


def test_valid_scenario_has_a_footprint(lib, scen):
    rc, b = footprint(lib, scen)
    assert rc == sim.OK and b > 0
    rc0, b0 = footprint(lib, scen, with_vehicles=False)
    assert rc0 == sim.OK and 0 < b0 < b


def test_route_offsets_are_checked_before_use(lib, scen):
    off = scen.route_off.copy()
    n = scen.n_veh
    assert footprint(lib, with_routes(scen, off))[0] == sim.OK
    bad = []
    a = off.copy()
    a[0] = 1                      # does not start at 0
    bad.append(a)
    a = off.copy()
    a[3] = a[2]                   # an empty route
    bad.append(a)
    a = off.copy()
    a[n] = a[n // 2]              # total below an earlier offset
    bad.append(a)
    a = off.copy()
    a[n] = -5                     # negative total
    bad.append(a)
    a = off.copy()
    a[1:] = a[1:][::-1]           # falling offsets
    bad.append(a)
    for a in bad:
        assert footprint(lib, with_routes(scen, a))[0] == sim.E_INVAL
    missing = dataclasses.replace(scen, route_off=None)
    assert footprint(lib, missing)[0] == sim.E_INVAL


def test_network_checks(lib, scen):
    def rc_of(**kw):
        return footprint(lib, dataclasses.replace(scen, **kw))[0]

    lanes = scen.link_lanes.copy()
    lanes[0] = 5
    assert rc_of(link_lanes=lanes) == sim.E_INVAL
    length = scen.link_len.copy()
    length[0] = scen.vmax           # shorter than vmax + 1 cells
    assert rc_of(link_len=length) == sim.E_INVAL
    to = scen.link_to.copy()
    to[0] = scen.link_from[0]       # a self-loop
    assert rc_of(link_to=to) == sim.E_INVAL
    to = scen.link_to.copy()
    to[0] = scen.n_nodes            # node out of range
    assert rc_of(link_to=to) == sim.E_INVAL
    # two links entering one node with the same rank
    node = scen.link_to[0]
    into = np.flatnonzero(scen.link_to == node)
    assert len(into) >= 2
    rank = scen.link_rank.copy()
    rank[into[1]] = rank[into[0]]
    assert rc_of(link_rank=rank) == sim.E_INVAL
    for bad in (np.nan, -1.0, np.inf):
        cost = np.ones(scen.n_links, np.float32)
        cost[7] = bad
        assert footprint(lib, scen, link_cost=cost)[0] == sim.E_INVAL
    assert footprint(lib, scen, link_cost=np.ones(scen.n_links, np.float32))[0] == sim.OK


def test_parameter_checks(lib, scen):
    for kw in ({"vmax": 0}, {"vmax": 8}):
        assert footprint(lib, dataclasses.replace(scen, **kw))[0] == sim.E_INVAL


def test_context_configuration_checks(lib):
    # sim_create checks its configuration before any device call, so these
    # are refused the same way with or without a GPU
    def create(**kw):
        f = dict(abi_version=sim.ABI_VERSION, max_slots=1, stream=None,
                 tile_lanes=0, back_pieces=0, graph_steps=0, step_mode=0,
                 tile_cells=0, reserved=0)
        f.update(kw)
        cfg = sim.sim_config(**f)
        h = C.c_void_p()
        rc = lib.sim_create(C.byref(cfg), C.byref(h))
        if rc == sim.OK:
            lib.sim_destroy(h)
        return rc

    assert create(abi_version=sim.ABI_VERSION + 1) == sim.E_ABI
    for kw in ({"max_slots": 0}, {"max_slots": 65537}, {"tile_lanes": -1},
               {"tile_lanes": 65}, {"back_pieces": 9}, {"back_pieces": -1},
               {"step_mode": 3}, {"step_mode": -1}, {"tile_cells": 63}, {"tile_cells": 65537},
               {"graph_steps": 4097}, {"reserved": 1}):
        assert create(**kw) == sim.E_INVAL, kw
    assert lib.sim_create(None, None) == sim.E_INVAL
