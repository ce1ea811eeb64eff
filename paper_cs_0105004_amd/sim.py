"""Python binding of libtransims (ctypes over the C ABI in include/transims.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of libtransims.so.  PyTorch provides the device workspace (a uint8
tensor per slot) and the stream.  There is no CPU fallback: if the library is
not built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtransims.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "transims.h")

ABI_VERSION = 3
OK, E_INVAL, E_NOMEM, E_STATE, E_DEVICE, E_CAPACITY, E_ABI = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "SIM_OK", -1: "SIM_E_INVAL", -2: "SIM_E_NOMEM",
                -3: "SIM_E_STATE", -4: "SIM_E_DEVICE", -5: "SIM_E_CAPACITY",
                -6: "SIM_E_ABI"}


class SimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class sim_config(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("max_slots", C.c_int32),
                ("stream", C.c_void_p), ("tile_lanes", C.c_int32),
                ("back_pieces", C.c_int32), ("graph_steps", C.c_int32),
                ("step_mode", C.c_int32), ("tile_cells", C.c_int32),
                ("reserved", C.c_int32)]


class sim_params(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("vmax", C.c_int32),
                ("slow_thr", C.c_uint64), ("lc_thr", C.c_uint64),
                ("lc_desp", C.c_int32), ("seed", C.c_uint64)]


class sim_network(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_links", C.c_int32),
                ("from_", C.c_void_p), ("to", C.c_void_p), ("len", C.c_void_p),
                ("lanes", C.c_void_p), ("rank", C.c_void_p),
                ("conn_off", C.c_void_p), ("conn_out", C.c_void_p),
                ("conn_lo", C.c_void_p), ("conn_hi", C.c_void_p),
                ("node_xy", C.c_void_p), ("link_cost", C.c_void_p),
                ("signal_plan", C.c_void_p), ("n_plans", C.c_int32),
                ("plan_cycle", C.c_void_p), ("plan_red", C.c_void_p),
                ("plan_offset", C.c_void_p)]


class sim_vehicles(C.Structure):
    _fields_ = [("n", C.c_int32), ("depart", C.c_void_p),
                ("route_off", C.c_void_p), ("route_links", C.c_void_p),
                ("init_status", C.c_void_p), ("init_lane", C.c_void_p),
                ("init_x", C.c_void_p), ("init_v", C.c_void_p),
                ("init_rptr", C.c_void_p), ("exit_t0", C.c_void_p),
                ("t0", C.c_int32)]


class sim_stats_t(C.Structure):
    _fields_ = [("t", C.c_int32), ("reserved", C.c_int32),
                ("n_waiting", C.c_int64), ("n_active", C.c_int64),
                ("n_arrived", C.c_int64), ("veh_updates", C.c_int64),
                ("sum_v", C.c_int64), ("crossings", C.c_int64),
                ("exits", C.c_int64), ("lane_changes", C.c_int64),
                ("insertions", C.c_int64), ("c_occ", C.c_int64),
                ("hash", C.c_uint64), ("dev_err", C.c_uint32),
                ("reserved2", C.c_uint32)]


class sim_kernel_time(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double)]


class sim_tiling(C.Structure):
    _fields_ = [("n_tiles", C.c_int32), ("n_lanes", C.c_int32),
                ("n_cells", C.c_int64), ("e_dmn", C.c_double),
                ("e_tile", C.c_double)]


_lib = None


def declared_symbols() -> list:
    """Names of the functions include/transims.h declares."""
    import re
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", text)))


def load_library() -> C.CDLL:
    """Loads libtransims.so (after torch, so that one HIP runtime serves
    both).  Raises if the library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libtransims.so is not built; run paper_cs_0105004_amd/build.py "
            "(or __graft_entry__.build())")
    import torch  # noqa: F401  (maps torch's libamdhip64 first)
    _lib = declare(C.CDLL(LIB_PATH))
    return _lib


def declare(L: C.CDLL) -> C.CDLL:
    """Declares the argument and result types of every entry point of a
    loaded libtransims."""
    vp, i32, u64p = C.c_void_p, C.c_int32, C.POINTER(C.c_uint64)
    L.sim_create.argtypes = [C.POINTER(sim_config), C.POINTER(vp)]
    L.sim_footprint.argtypes = [vp, C.POINTER(sim_params),
                                C.POINTER(sim_network), C.POINTER(sim_vehicles),
                                u64p]
    L.sim_load_network.argtypes = [vp, i32, C.POINTER(sim_params),
                                   C.POINTER(sim_network), vp, C.c_uint64]
    L.sim_load_vehicles.argtypes = [vp, i32, C.POINTER(sim_vehicles)]
    L.sim_step.argtypes = [vp, C.POINTER(i32), i32, i32]
    L.sim_step_noalloc.argtypes = [vp, C.POINTER(i32), i32, i32]
    L.sim_stats.argtypes = [vp, i32, C.POINTER(sim_stats_t)]
    L.sim_read_state.argtypes = [vp, i32] + [vp] * 7
    L.sim_link_costs.argtypes = [vp, i32, vp]
    L.sim_tiling_info.argtypes = [vp, i32, C.POINTER(sim_tiling)]
    L.sim_unload.argtypes = [vp, i32]
    L.sim_destroy.argtypes = [vp]
    L.sim_profile.argtypes = [vp, i32]
    L.sim_kernel_times.argtypes = [vp, C.POINTER(sim_kernel_time)]
    L.sim_last_error.argtypes = [vp]
    L.sim_last_error.restype = C.c_char_p
    for name in declared_symbols():
        if name != "sim_last_error":
            getattr(L, name).restype = C.c_int
    return L


def _p(a) -> Optional[int]:
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype)


class _Inputs:
    """ctypes structs for one scenario plus the arrays they point into."""

    def __init__(self, scen, link_cost=None):
        keep = []

        def k(a, dt):
            a = _c(a, dt)
            keep.append(a)
            return _p(a)

        self.params = sim_params(scen.flags, scen.vmax, scen.slow_thr,
                                 scen.lc_thr, scen.lc_desp,
                                 scen.seed & 0xFFFFFFFFFFFFFFFF)
        self.net = sim_network(
            scen.n_nodes, scen.n_links, k(scen.link_from, np.int32),
            k(scen.link_to, np.int32), k(scen.link_len, np.int32),
            k(scen.link_lanes, np.int8), k(scen.link_rank, np.int8),
            k(scen.conn_off, np.int64), k(scen.conn_out, np.int32),
            k(scen.conn_lo, np.int8), k(scen.conn_hi, np.int8),
            k(None if scen.node_xy is None else scen.node_xy.ravel(),
              np.float64),
            k(link_cost, np.float32), k(scen.signal_plan, np.int8),
            0 if scen.plan_cycle is None else len(scen.plan_cycle),
            k(scen.plan_cycle, np.int32), k(scen.plan_red, np.int32),
            k(scen.plan_offset, np.int32))
        self.veh = sim_vehicles(
            scen.n_veh, k(scen.depart, np.int32), k(scen.route_off, np.int64),
            k(scen.route_links, np.int32), k(scen.init_status, np.int8),
            k(scen.init_lane, np.int8), k(scen.init_x, np.int32),
            k(scen.init_v, np.int8), k(scen.init_rptr, np.int32),
            k(scen.exit_t0, np.int32), scen.t0)
        self._keep = keep


class Context:
    """A libtransims context on the current GPU with `max_slots` slots."""

    def __init__(self, max_slots: int = 1, tile_lanes: int = 0,
                 back_pieces: int = 0, graph_steps: int = 0, stream=None,
                 step_mode: int = 0, tile_cells: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libtransims needs a GPU; none is visible")
        self.lib = load_library()
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        cfg = sim_config(ABI_VERSION, max_slots, C.c_void_p(stream.cuda_stream),
                         tile_lanes, back_pieces, graph_steps, step_mode,
                         tile_cells, 0)
        h = C.c_void_p()
        self._check(self.lib.sim_create(C.byref(cfg), C.byref(h)), None)
        self.h = h
        self.max_slots = max_slots
        self.ws: Dict[int, object] = {}
        self.scen: Dict[int, object] = {}

    def _check(self, rc: int, h=Ellipsis):
        if rc != OK:
            hh = self.h if h is Ellipsis else h
            msg = self.lib.sim_last_error(hh).decode() if hh else ""
            raise SimError(rc, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.sim_destroy(self.h)
            self.h = None
            self.ws.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, scen) -> int:
        inp = _Inputs(scen)
        b = C.c_uint64()
        self._check(self.lib.sim_footprint(self.h, C.byref(inp.params),
                                           C.byref(inp.net), C.byref(inp.veh),
                                           C.byref(b)))
        return int(b.value)

    def load(self, slot: int, scen, link_cost=None, ws=None):
        """Allocates the slot's workspace (unless given) and loads scen.  If
        the library refuses the network or the vehicles, the slot is left
        empty (a scenario loaded there before is gone too) and SimError is
        raised."""
        inp = _Inputs(scen, link_cost)
        if ws is None:
            ws = self.torch.empty(self.footprint(scen), dtype=self.torch.uint8,
                                  device="cuda")
        rc = self.lib.sim_load_network(
            self.h, slot, C.byref(inp.params), C.byref(inp.net),
            C.c_void_p(ws.data_ptr()), ws.numel())
        if rc == OK:
            # the slot points into ws from here on: keep ws alive with it
            self.ws[slot], self.scen[slot] = ws, scen
            rc = self.lib.sim_load_vehicles(self.h, slot, C.byref(inp.veh))
            if rc == OK:
                return
        msg = (self.lib.sim_last_error(self.h) or b"").decode()
        if 0 <= slot < self.max_slots:
            # never leave the library pointing into a workspace that the
            # binding no longer holds
            self.lib.sim_unload(self.h, slot)
            self.ws.pop(slot, None)
            self.scen.pop(slot, None)
        raise SimError(rc, msg)

    def step(self, slots, n_steps: int = 1):
        if isinstance(slots, int):
            slots = [slots]
        arr = (C.c_int32 * len(slots))(*slots)
        self._check(self.lib.sim_step(self.h, arr, len(slots), int(n_steps)))

    def step_noalloc(self, slots, n_steps: int = 1):
        """sim_step_noalloc: the same steps without any device allocation
        (the work list goes to the library's fixed device scratch)."""
        if isinstance(slots, int):
            slots = [slots]
        arr = (C.c_int32 * len(slots))(*slots)
        self._check(self.lib.sim_step_noalloc(self.h, arr, len(slots),
                                              int(n_steps)))

    def stats(self, slot: int = 0) -> dict:
        s = sim_stats_t()
        rc = self.lib.sim_stats(self.h, slot, C.byref(s))
        out = {name: getattr(s, name) for name, _ in sim_stats_t._fields_
               if not name.startswith("reserved")}
        self._check(rc)
        return out

    def state(self, slot: int = 0) -> dict:
        scen = self.scen[slot]
        n = scen.n_veh
        out = dict(status=np.zeros(n, np.int8), link=np.zeros(n, np.int32),
                   lane=np.zeros(n, np.int8), x=np.zeros(n, np.int32),
                   v=np.zeros(n, np.int8), rptr=np.zeros(n, np.int32),
                   exit_t=np.zeros(scen.n_route_entries, np.int32))
        self._check(self.lib.sim_read_state(
            self.h, slot, *[C.c_void_p(_p(out[k])) for k in
                            ("status", "link", "lane", "x", "v", "rptr",
                             "exit_t")]))
        return out

    def link_costs(self, slot: int = 0) -> np.ndarray:
        out = np.zeros(self.scen[slot].n_links, np.float32)
        self._check(self.lib.sim_link_costs(self.h, slot,
                                            C.c_void_p(_p(out))))
        return out

    def tiling(self, slot: int = 0) -> dict:
        t = sim_tiling()
        self._check(self.lib.sim_tiling_info(self.h, slot, C.byref(t)))
        return {name: getattr(t, name) for name, _ in sim_tiling._fields_}

    def profile(self, enable: bool = True):
        """Brackets every kernel launch with HIP events (kernel timing)."""
        self._check(self.lib.sim_profile(self.h, int(bool(enable))))

    def kernel_times(self) -> dict:
        """{kind: (launches, total_ms)} since the last call; waits."""
        arr = (sim_kernel_time * 4)()
        self._check(self.lib.sim_kernel_times(self.h, arr))
        return {name: (arr[k].launches, arr[k].total_ms)
                for k, name in enumerate(("front", "back", "ring", "step"))}

    def unload(self, slot: int):
        self._check(self.lib.sim_unload(self.h, slot))
        self.ws.pop(slot, None)
        self.scen.pop(slot, None)
