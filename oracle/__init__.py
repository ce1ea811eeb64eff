"""CPU oracle for the TRANSIMS cellular-automaton step -- TEST INFRASTRUCTURE.

A ctypes binding over the plain C implementation in transims_oracle.c.  Only
the tests, the smoke entry point and the CPU-baseline leg of the benchmark
may import this package; the GPU library never does, and this package never
loads the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "transims_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libtransims_oracle.so")

WAITING, ACTIVE, ARRIVED = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libtransims_oracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra",
                               "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("vmax", C.c_int32),
                ("slow_thr", C.c_uint64), ("lc_thr", C.c_uint64),
                ("lc_desp", C.c_int32), ("seed", C.c_uint64)]


class _Network(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_links", C.c_int32),
                ("from_", C.c_void_p), ("to", C.c_void_p),
                ("len", C.c_void_p), ("lanes", C.c_void_p),
                ("rank", C.c_void_p), ("conn_off", C.c_void_p),
                ("conn_out", C.c_void_p), ("conn_lo", C.c_void_p),
                ("conn_hi", C.c_void_p), ("signal_plan", C.c_void_p),
                ("n_plans", C.c_int32), ("plan_cycle", C.c_void_p),
                ("plan_red", C.c_void_p), ("plan_offset", C.c_void_p)]


class _Vehicles(C.Structure):
    _fields_ = [("n", C.c_int32), ("depart", C.c_void_p),
                ("route_off", C.c_void_p), ("route_links", C.c_void_p),
                ("init_status", C.c_void_p), ("init_lane", C.c_void_p),
                ("init_x", C.c_void_p), ("init_v", C.c_void_p),
                ("init_rptr", C.c_void_p), ("exit_t0", C.c_void_p),
                ("t0", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("t", C.c_int32), ("n_waiting", C.c_int64),
                ("n_active", C.c_int64), ("n_arrived", C.c_int64),
                ("veh_updates", C.c_int64), ("sum_v", C.c_int64),
                ("crossings", C.c_int64), ("exits", C.c_int64),
                ("lane_changes", C.c_int64), ("insertions", C.c_int64),
                ("c_occ", C.c_int64), ("hash", C.c_uint64)]


_lib = None


def bind(path: str) -> C.CDLL:
    """Loads an oracle library built from transims_oracle.c at `path` and
    declares its signatures."""
    L = C.CDLL(path)
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [C.POINTER(_Params), C.POINTER(_Network),
                             C.POINTER(_Vehicles), C.c_char_p, C.c_int]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_step.argtypes = [C.c_void_p, C.c_int32]
    L.orc_step.restype = C.c_int
    L.orc_get_stats.argtypes = [C.c_void_p, C.POINTER(_Stats)]
    L.orc_get_state.argtypes = [C.c_void_p] + [C.c_void_p] * 7
    L.orc_philox4x32_10.argtypes = [C.c_void_p] * 3
    L.orc_philox4x64_10.argtypes = [C.c_void_p] * 3
    L.orc_mix64.argtypes = [C.c_uint64]
    L.orc_mix64.restype = C.c_uint64
    return L


def lib():
    """The oracle library: oracle/libtransims_oracle.so, rebuilt when its
    source is newer; a test that runs the pins against a planted mistake
    names a mutant build in TRANSIMS_ORACLE_LIB instead."""
    global _lib
    if _lib is None:
        mutant = os.environ.get("TRANSIMS_ORACLE_LIB")
        if mutant:
            _lib = bind(mutant)
        else:
            if not os.path.exists(_LIB_PATH) or (
                    os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
                build()
            _lib = bind(_LIB_PATH)
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _arr(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype)


class OracleError(RuntimeError):
    pass


class OracleSim:
    """One scenario on the CPU oracle.  `scen` is a scenarios.Scenario."""

    def __init__(self, scen):
        self.scen = scen
        self._keep = []

        def k(a, dt):
            a = _arr(a, dt)
            self._keep.append(a)
            return _ptr(a)

        p = _Params(scen.flags, scen.vmax, scen.slow_thr, scen.lc_thr,
                    scen.lc_desp, scen.seed)
        net = _Network(scen.n_nodes, scen.n_links, k(scen.link_from, np.int32),
                       k(scen.link_to, np.int32), k(scen.link_len, np.int32),
                       k(scen.link_lanes, np.int8), k(scen.link_rank, np.int8),
                       k(scen.conn_off, np.int64), k(scen.conn_out, np.int32),
                       k(scen.conn_lo, np.int8), k(scen.conn_hi, np.int8),
                       k(scen.signal_plan, np.int8),
                       0 if scen.plan_cycle is None else len(scen.plan_cycle),
                       k(scen.plan_cycle, np.int32), k(scen.plan_red, np.int32),
                       k(scen.plan_offset, np.int32))
        veh = _Vehicles(scen.n_veh, k(scen.depart, np.int32),
                        k(scen.route_off, np.int64),
                        k(scen.route_links, np.int32),
                        k(scen.init_status, np.int8),
                        k(scen.init_lane, np.int8), k(scen.init_x, np.int32),
                        k(scen.init_v, np.int8), k(scen.init_rptr, np.int32),
                        k(scen.exit_t0, np.int32), scen.t0)
        err = C.create_string_buffer(512)
        h = lib().orc_create(C.byref(p), C.byref(net), C.byref(veh), err, 512)
        self._keep = []
        if not h:
            raise OracleError(err.value.decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    __del__ = close

    def step(self, n: int = 1):
        if lib().orc_step(self._h, int(n)) != 0:
            raise OracleError("oracle invariant broken (two vehicles in a cell)")

    def stats(self) -> dict:
        s = _Stats()
        lib().orc_get_stats(self._h, C.byref(s))
        return {name: getattr(s, name) for name, _ in _Stats._fields_}

    def state(self) -> dict:
        n = self.scen.n_veh
        out = dict(status=np.zeros(n, np.int8), link=np.zeros(n, np.int32),
                   lane=np.zeros(n, np.int8), x=np.zeros(n, np.int32),
                   v=np.zeros(n, np.int8), rptr=np.zeros(n, np.int32))
        R = self.scen.n_route_entries
        out["exit_t"] = np.zeros(R, np.int32)
        lib().orc_get_state(self._h, *[_ptr(out[k]) for k in
                                       ("status", "link", "lane", "x", "v",
                                        "rptr", "exit_t")])
        return out


def philox4x32_10(ctr, key):
    """Philox4x32-10 of one 4-word counter under a 2-word key."""
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    o = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def mix64(z: int) -> int:
    return int(lib().orc_mix64(C.c_uint64(z)))
