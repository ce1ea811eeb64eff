"""The Python binding's bookkeeping around the C ABI, on the CPU with a
stand-in for the library: a slot that the library refers to always has
its workspace held by the binding, and a refused load leaves the slot
empty."""
import ctypes as C

import pytest

from paper_cs_0105004_amd import scenarios as S
from paper_cs_0105004_amd import sim


class FakeLib:
    """Records calls; returns the given status for each loader."""

    def __init__(self, net_rc=sim.OK, veh_rc=sim.OK):
        self.net_rc, self.veh_rc, self.calls = net_rc, veh_rc, []

    def sim_load_network(self, h, slot, p, net, ws, nbytes):
        self.calls.append(("network", slot, ws.value, nbytes))
        return self.net_rc

    def sim_load_vehicles(self, h, slot, veh):
        self.calls.append(("vehicles", slot))
        return self.veh_rc

    def sim_unload(self, h, slot):
        self.calls.append(("unload", slot))
        return sim.OK

    def sim_last_error(self, h):
        return b"refused"

    def sim_destroy(self, h):
        return sim.OK


class FakeWorkspace:
    def __init__(self, ptr):
        self.ptr = ptr

    def data_ptr(self):
        return self.ptr

    def numel(self):
        return 1 << 20


def context(lib):
    ctx = object.__new__(sim.Context)  # no GPU: the constructor is bypassed
    ctx.lib, ctx.h, ctx.max_slots = lib, C.c_void_p(1), 2
    ctx.ws, ctx.scen = {}, {}
    return ctx


@pytest.fixture(scope="module")
def scen():
    return S.portland_like(scale=0.01, T=50, seed=3)


def test_load_keeps_the_workspace_with_the_slot(scen):
    lib = FakeLib()
    ctx = context(lib)
    ws = FakeWorkspace(4096)
    ctx.load(1, scen, ws=ws)
    assert ctx.ws[1] is ws and ctx.scen[1] is scen
    assert lib.calls == [("network", 1, 4096, 1 << 20), ("vehicles", 1)]
    ws2 = FakeWorkspace(8192)
    ctx.load(1, scen, ws=ws2)  # reload: the new workspace replaces the old
    assert ctx.ws[1] is ws2


@pytest.mark.parametrize("net_rc,veh_rc", [(sim.OK, sim.E_INVAL),
                                           (sim.E_NOMEM, sim.OK)])
def test_refused_load_leaves_the_slot_empty(scen, net_rc, veh_rc):
    lib = FakeLib()
    ctx = context(lib)
    ctx.load(0, scen, ws=FakeWorkspace(4096))
    lib.net_rc, lib.veh_rc = net_rc, veh_rc
    with pytest.raises(sim.SimError) as e:
        ctx.load(0, scen, ws=FakeWorkspace(8192))
    assert e.value.code == (veh_rc if net_rc == sim.OK else net_rc)
    assert "refused" in str(e.value)
    assert lib.calls[-1] == ("unload", 0)
    assert 0 not in ctx.ws and 0 not in ctx.scen
