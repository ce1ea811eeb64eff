"""The library's host code on the CPU: transims.cpp and tiler.cpp built into
a host-only library against tests/helpers/hip_stub.cpp, a stand-in for the
HIP runtime whose kernels do nothing.  No step is computed here; what runs
is the real code of the C ABI around the kernels: argument checks that
need a loaded slot, slot bookkeeping, tiling, workspace carving, and the
uploads and copies back."""
import ctypes as C
import dataclasses
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_cs_0105004_amd import scenarios as S
from paper_cs_0105004_amd import sim

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_cs_0105004_amd", "csrc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    cxx = shutil.which("clang++", path="/opt/rocm/llvm/bin") or \
        shutil.which("amdclang++")
    if not cxx:
        pytest.skip("no ROCm clang++")
    out = str(tmp_path_factory.mktemp("host") / "libtransims_host.so")
    subprocess.check_call(
        [cxx, "-std=c++17", "-O1", "-fPIC", "-shared", "-Wl,-Bsymbolic",
         "-Wl,--no-undefined", "-D__HIP_PLATFORM_AMD__",
         "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
         "-I" + CSRC, os.path.join(CSRC, "transims.cpp"),
         os.path.join(CSRC, "tiler.cpp"),
         os.path.join(HERE, "helpers", "hip_stub.cpp"), "-o", out])
    return sim.declare(C.CDLL(out))


class Host:
    """A context of the host-only library; workspaces are numpy buffers."""

    def __init__(self, lib, max_slots=2, **cfg):
        self.lib = lib
        f = dict(abi_version=sim.ABI_VERSION, max_slots=max_slots,
                 stream=None, tile_lanes=0, back_pieces=0, graph_steps=0,
                 step_mode=0, tile_cells=0, reserved=0)
        f.update(cfg)
        self.h = C.c_void_p()
        assert lib.sim_create(C.byref(sim.sim_config(**f)),
                              C.byref(self.h)) == sim.OK
        self.keep = {}

    def err(self):
        return self.lib.sim_last_error(self.h).decode()

    def footprint(self, scen, vehicles=True):
        inp = sim._Inputs(scen)
        b = C.c_uint64()
        assert self.lib.sim_footprint(
            self.h, C.byref(inp.params), C.byref(inp.net),
            C.byref(inp.veh) if vehicles else None, C.byref(b)) == sim.OK
        return b.value

    def load_network(self, slot, scen, nbytes=None, link_cost=None):
        inp = sim._Inputs(scen, link_cost)
        nbytes = self.footprint(scen) if nbytes is None else nbytes
        ws = np.zeros(nbytes + 256, np.uint8)
        ptr = (ws.ctypes.data + 255) // 256 * 256
        self.keep[slot] = (ws, inp)
        return self.lib.sim_load_network(self.h, slot, C.byref(inp.params),
                                         C.byref(inp.net), C.c_void_p(ptr),
                                         nbytes)

    def load_vehicles(self, slot, scen):
        inp = sim._Inputs(scen)
        self.keep[(slot, "v")] = inp
        return self.lib.sim_load_vehicles(self.h, slot, C.byref(inp.veh))

    def step(self, slots, n):
        arr = (C.c_int32 * len(slots))(*slots)
        return self.lib.sim_step(self.h, arr, len(slots), n)

    def tiling(self, slot):
        t = sim.sim_tiling()
        rc = self.lib.sim_tiling_info(self.h, slot, C.byref(t))
        return rc, t

    def exit_times(self, slot, n_route):
        out = np.full(n_route, -7, np.int32)
        rc = self.lib.sim_read_state(self.h, slot, None, None, None, None,
                                     None, None, C.c_void_p(out.ctypes.data))
        return rc, out

    def close(self):
        self.lib.sim_destroy(self.h)


@pytest.fixture(scope="module")
def grid():
    return S.portland_like(scale=0.05, T=200, depart_max=100, seed=17)


@pytest.fixture(scope="module")
def lc_grid():
    return S.portland_like(scale=0.05, T=200, depart_max=100, seed=18,
                           flags=S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES)


@pytest.fixture(scope="module")
def midrun(grid):
    """grid after 120 oracle steps: active vehicles and set exit times."""
    o = oracle.OracleSim(grid)
    o.step(120)
    state = o.state()
    o.close()
    return grid.with_state(state, 120)


def test_load_and_tiling(lib, grid, lc_grid):
    h = Host(lib)
    for slot, scen in ((0, grid), (1, lc_grid)):
        assert h.load_network(slot, scen) == sim.OK, h.err()
        assert h.load_vehicles(slot, scen) == sim.OK, h.err()
        rc, t = h.tiling(slot)
        assert rc == sim.OK
        assert t.n_lanes == int(scen.link_lanes.sum())
        assert t.n_cells == int((scen.link_len * scen.link_lanes.astype(np.int64)).sum())
        assert 0 < t.n_tiles <= t.n_lanes
        assert 0 < t.e_tile <= 1 and 0 < t.e_dmn <= 1
    assert h.step([0, 1], 70) == sim.OK  # graphs of 64 steps + 6 launches
    h.close()


def test_footprint_is_enough_and_needed(lib, grid):
    h = Host(lib)
    need = h.footprint(grid)
    assert h.load_network(0, grid, nbytes=need) == sim.OK
    assert h.load_vehicles(0, grid) == sim.OK
    # a workspace that holds the network but not the vehicles
    net_only = h.footprint(grid, vehicles=False)
    assert net_only < need
    assert h.load_network(0, grid, nbytes=net_only) == sim.OK
    assert h.load_vehicles(0, grid) == sim.E_NOMEM
    assert h.load_network(0, grid, nbytes=net_only // 2) == sim.E_NOMEM
    h.close()


def test_exit_times_round_trip_in_route_order(lib, midrun):
    assert (midrun.exit_t0 >= 0).sum() > 100
    h = Host(lib)
    assert h.load_network(0, midrun) == sim.OK
    assert h.load_vehicles(0, midrun) == sim.OK, h.err()
    rc, got = h.exit_times(0, midrun.n_route_entries)
    assert rc == sim.OK
    np.testing.assert_array_equal(got, midrun.exit_t0)
    h.close()


def broken(scen, **arrays):
    s = dataclasses.replace(scen)
    for k, v in arrays.items():
        setattr(s, k, v)
    return s


def test_vehicle_checks_that_need_a_loaded_network(lib, midrun, lc_grid):
    m = midrun
    act = np.flatnonzero(m.init_status == S.ACTIVE)
    link_of = m.route_links[m.route_off[act] + m.init_rptr[act]]
    # two active vehicles on one link
    vals, counts = np.unique(link_of, return_counts=True)
    shared = vals[counts >= 2][0]
    a, b = (int(i) for i in act[link_of == shared][:2])
    link_a = shared

    def with_(arr, i, val):
        arr = arr.copy()
        arr[i] = val
        return arr

    cases = {
        "cell past the link end": broken(m, init_x=with_(m.init_x, a, m.link_len[link_a])),
        "negative cell": broken(m, init_x=with_(m.init_x, a, -1)),
        "lane out of range": broken(m, init_lane=with_(m.init_lane, a, m.link_lanes[link_a])),
        "speed above vmax": broken(m, init_v=with_(m.init_v, a, m.vmax + 1)),
        "route pointer past the route": broken(
            m, init_rptr=with_(m.init_rptr, a, m.route_off[a + 1] - m.route_off[a])),
        "unknown status": broken(m, init_status=with_(m.init_status, a, 3)),
        "negative first step": broken(m, t0=-1),
    }
    # two vehicles on one cell: b placed where a is
    cases["two vehicles on one cell"] = broken(
        m, init_lane=with_(m.init_lane, b, m.init_lane[a]),
        init_x=with_(m.init_x, b, m.init_x[a]))
    # a route whose consecutive links do not meet
    rl = m.route_links.copy()
    i = int(np.flatnonzero(np.diff(m.route_off) >= 2)[0])
    j = m.route_off[i] + 1
    bad = np.flatnonzero(m.link_from != m.link_to[rl[j - 1]])[0]
    rl[j] = bad
    cases["route links not connected"] = broken(m, route_links=rl)
    rl = m.route_links.copy()
    rl[0] = m.n_links
    cases["route link out of range"] = broken(m, route_links=rl)
    # a departure beyond the packed field
    waiting = np.flatnonzero(m.init_status == S.WAITING)
    assert len(waiting) > 0
    cases["departure too late"] = broken(
        m, depart=with_(m.depart, int(waiting[0]), 1 << 27))
    # a turn the lane table does not list
    lc = lc_grid
    conn_out = lc.conn_out.copy()
    first = lc.route_links[lc.route_off[0]]
    nxt = lc.route_links[lc.route_off[0] + 1]
    k = [e for e in range(lc.conn_off[first], lc.conn_off[first + 1])
         if lc.conn_out[e] == nxt]
    assert k
    others = [o for o in np.flatnonzero(lc.link_from == lc.link_to[first])
              if o != nxt and o not in lc.conn_out[lc.conn_off[first]:lc.conn_off[first + 1]]]
    h = Host(lib)
    for name, scen in cases.items():
        assert h.load_network(0, scen) == sim.OK, name
        assert h.load_vehicles(0, scen) == sim.E_INVAL, name
        # a refused load leaves the slot without vehicles
        assert h.step([0], 1) == sim.E_STATE, name
    assert others
    conn_out[k[0]] = others[0]  # the turn now leads elsewhere
    scen = broken(lc, conn_out=conn_out)
    assert h.load_network(0, scen) == sim.OK
    assert h.load_vehicles(0, scen) == sim.E_INVAL
    h.close()


def test_slot_bookkeeping(lib, grid):
    h = Host(lib, max_slots=3)
    assert h.step([0], 1) == sim.E_STATE            # nothing loaded
    assert h.load_network(0, grid) == sim.OK
    assert h.step([0], 1) == sim.E_STATE            # network only
    assert h.load_vehicles(0, grid) == sim.OK
    assert h.step([0], 5) == sim.OK
    assert h.step([0, 0], 1) == sim.E_INVAL         # listed twice
    assert h.step([0], -1) == sim.E_INVAL
    assert h.step([3], 1) == sim.E_INVAL            # out of range
    # a refused network leaves the slot empty, whatever was loaded before
    bad = broken(grid, vmax=9)
    assert h.load_network(0, bad, nbytes=1 << 20) == sim.E_INVAL
    assert h.step([0], 1) == sim.E_STATE
    assert h.tiling(0)[0] == sim.E_STATE
    # the step index must not overflow
    late = broken(grid, t0=(1 << 31) - 10)
    assert h.load_network(1, late) == sim.OK
    assert h.load_vehicles(1, late) == sim.OK
    assert h.step([1], 100) == sim.E_CAPACITY
    assert h.lib.sim_unload(h.h, 1) == sim.OK
    assert h.step([1], 1) == sim.E_STATE
    h.close()


def test_link_costs_shape_the_tiles(lib, grid):
    h = Host(lib)
    assert h.load_network(0, grid) == sim.OK
    base = h.tiling(0)[1].n_tiles
    cost = np.ones(grid.n_links, np.float32)
    cost[: grid.n_links // 10] = 50.0   # a tenth of the links cost far more
    assert h.load_network(0, grid, link_cost=cost) == sim.OK
    rc, t = h.tiling(0)
    assert rc == sim.OK and t.n_tiles > base
    h.close()


def test_lane_change_tiles_ordered_only_between_limits(lib):
    # a graph of the two-kernel step starts with the tile-ordering kernel
    # exactly when its list holds more lane-change tiles than are resident
    # at once (6,144) and no more than its eight workgroups, one per XCD,
    # sort (8 x 2,048); the one-kernel step is never reordered
    lib.stub_order_nodes.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.stub_order_nodes.restype = C.c_int
    last_n, grid = C.c_int(), C.c_int()
    lc = S.FLAG_LANE_CHANGE | S.FLAG_TURN_LANES
    regions = set()
    for scale, flags in ((0.1, lc), (0.35, lc), (0.9, lc), (0.35, 0)):
        scen = S.portland_like(scale=scale, T=50, depart_max=10, seed=23,
                               flags=flags)
        h = Host(lib, max_slots=1, tile_lanes=1, tile_cells=64,
                 graph_steps=8)  # one link per tile
        assert h.load_network(0, scen) == sim.OK, h.err()
        assert h.load_vehicles(0, scen) == sim.OK, h.err()
        n = h.tiling(0)[1].n_tiles
        lib.stub_order_nodes(C.byref(last_n), C.byref(grid))
        assert h.step([0], 8) == sim.OK, h.err()  # one graph of 8 steps
        k = lib.stub_order_nodes(C.byref(last_n), C.byref(grid))
        if flags and 6144 < n <= 8 * 2048:
            assert (k, last_n.value, grid.value) == (1, n, 8), (scale, n)
        else:
            assert k == 0, (scale, flags, n)
        regions.add((bool(flags), (n > 6144) + (n > 8 * 2048)))
        h.close()
    assert regions == {(True, 0), (True, 1), (True, 2), (False, 1)}, regions


def test_ring_mode_checks(lib):
    h = Host(lib)
    ring = S.ring()
    assert h.load_network(0, ring) == sim.OK, h.err()
    assert h.load_vehicles(0, ring) == sim.OK, h.err()
    assert h.step([0], 10) == sim.OK

    def with_(name, i, val):
        arr = getattr(ring, name).copy()
        arr[i] = val
        return broken(ring, **{name: arr})

    bad = {
        "cell past the ring": with_("init_x", 3, ring.link_len[0]),
        "negative cell": with_("init_x", 3, -1),
        "two vehicles on one cell": with_("init_x", 3, ring.init_x[4]),
        "speed above vmax": with_("init_v", 3, ring.vmax + 1),
        "other lane": with_("init_lane", 3, 1),
        "not on the ring": with_("init_status", 3, S.WAITING),
        "no placement": broken(ring, init_status=None),
    }
    for name, scen in bad.items():
        assert h.load_network(0, scen, nbytes=1 << 20) == sim.OK, name
        assert h.load_vehicles(0, scen) == sim.E_INVAL, name
        assert h.step([0], 1) == sim.E_STATE, name
    # the ring keeps its vehicles in LDS: at most 4096
    crowded = S.ring(L=8000, n=4097)
    assert h.load_network(0, crowded, nbytes=1 << 20) == sim.OK
    assert h.load_vehicles(0, crowded) == sim.E_CAPACITY
    # a ring is one single-lane link of 1..32767 cells
    for kw in ({"link_len": np.array([32768], np.int32)},
               {"link_lanes": np.array([2], np.int8)}):
        assert h.load_network(0, broken(ring, **kw), nbytes=1 << 20) == sim.E_INVAL
    h.close()


@pytest.mark.parametrize("graph_steps", [0, 16, -1])
def test_kernel_time_bookkeeping(lib, grid, lc_grid, graph_steps):
    # profiled steps: graphs of graph_steps steps with event nodes between
    # the kernels (and a graph of its own for the remainder), or launches
    # bracketed by events; every launch is counted under its kernel kind
    h = Host(lib, max_slots=2, graph_steps=graph_steps)
    assert h.load_network(0, grid) == sim.OK and h.load_vehicles(0, grid) == sim.OK
    assert h.load_network(1, lc_grid) == sim.OK and h.load_vehicles(1, lc_grid) == sim.OK
    assert h.lib.sim_profile(h.h, 1) == sim.OK
    for slots, n in (([0], 70), ([1], 70), ([0, 1], 37)):
        assert h.step(slots, n) == sim.OK
    kt = (sim.sim_kernel_time * 4)()
    assert h.lib.sim_kernel_times(h.h, kt) == sim.OK
    launches = {name: kt[k].launches
                for k, name in enumerate(("front", "back", "ring", "step"))}
    # slot 0 takes one kernel per step, slot 1 two; together, one of each
    assert launches == {"front": 70 + 37, "back": 70 + 37, "ring": 0,
                        "step": 70 + 37}
    # the sums start again after a read
    assert h.lib.sim_kernel_times(h.h, kt) == sim.OK
    assert all(kt[k].launches == 0 for k in range(4))
    h.close()


def test_c_example_builds_and_runs(lib, tmp_path):
    # the C usage example compiles as plain C11 against the header and runs
    # every call of its sequence with SIM_OK (against the host-only library)
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("no gcc")
    libdir = os.path.dirname(lib._name)
    exe = str(tmp_path / "c_example")
    subprocess.check_call(
        [gcc, "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
         "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include",
         os.path.join(HERE, "helpers", "c_example.c"),
         lib._name, "-Wl,-rpath," + libdir, "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("t 20,")


def test_step_noalloc_bookkeeping(lib, grid):
    """The allocation-free step checks its slot list like sim_step, advances
    the listed slots, and refuses more slots than its fixed scratch holds
    before enqueuing anything."""
    h = Host(lib, max_slots=3)

    def noalloc(slots, n):
        arr = (C.c_int32 * len(slots))(*slots)
        return lib.sim_step_noalloc(h.h, arr, len(slots), n)

    assert noalloc([0], 1) == sim.E_STATE
    assert h.load_network(0, grid) == sim.OK
    assert h.load_vehicles(0, grid) == sim.OK
    assert noalloc([0], 5) == sim.OK
    assert noalloc([0, 0], 1) == sim.E_INVAL
    assert noalloc([0], -1) == sim.E_INVAL
    assert noalloc([3], 1) == sim.E_INVAL
    st = sim.sim_stats_t()
    assert lib.sim_stats(h.h, 0, C.byref(st)) == sim.OK and st.t == 5
    h.close()
    # one more ring slot than the scratch's slot list holds
    n = (1 << 14) + 1
    h = Host(lib, max_slots=n)
    ring = S.ring(2, 1, 1, "0", seed=1)
    inp = sim._Inputs(ring)
    ws = np.zeros(h.footprint(ring) * n + 256 * n, np.uint8)
    base = (ws.ctypes.data + 255) // 256 * 256
    per = (h.footprint(ring) + 255) // 256 * 256
    for k in range(n):
        assert lib.sim_load_network(h.h, k, C.byref(inp.params),
                                    C.byref(inp.net),
                                    C.c_void_p(base + k * per), per) == sim.OK
        assert lib.sim_load_vehicles(h.h, k, C.byref(inp.veh)) == sim.OK
    assert noalloc(list(range(n)), 1) == sim.E_CAPACITY
    assert "scratch" in h.err()
    assert lib.sim_stats(h.h, 0, C.byref(st)) == sim.OK and st.t == 0
    assert noalloc(list(range(n - 1)), 1) == sim.OK
    h.close()
