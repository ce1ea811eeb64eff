"""CPU-side checks of the C ABI: the library builds, loads next to torch's
HIP runtime, exports every function include/transims.h declares, and refuses
to run without a GPU (there is no CPU fallback)."""
import os
import subprocess
import sys

import pytest

from paper_cs_0105004_amd import sim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sim.LIB_PATH):
        from paper_cs_0105004_amd import build
        build.build()
    return sim.load_library()


def test_header_declares_the_boundary():
    names = sim.declared_symbols()
    for required in ("sim_create", "sim_footprint", "sim_load_network",
                     "sim_load_vehicles", "sim_step", "sim_stats",
                     "sim_read_state", "sim_unload", "sim_destroy",
                     "sim_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in sim.declared_symbols():
        assert hasattr(lib, name), name


def test_one_hip_runtime_in_process(lib):
    code = ("import torch, ctypes; ctypes.CDLL(%r); "
            "maps=open('/proc/self/maps').read(); "
            "libs={l.split()[-1] for l in maps.splitlines() "
            "if 'libamdhip64' in l}; print(len(libs)); print(libs)"
            % sim.LIB_PATH)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True,
                         text=True, check=True).stdout.split("\n")
    assert out[0].strip() == "1", out


def test_no_gpu_no_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        sim.Context()


def test_struct_layouts_match_header():
    import ctypes as C
    assert C.sizeof(sim.sim_config) == 40
    assert C.sizeof(sim.sim_params) == 40
    assert C.sizeof(sim.sim_stats_t) == 8 + 10 * 8 + 8 + 8
    assert C.sizeof(sim.sim_tiling) == 32


def test_struct_sizes_against_c_compiler(tmp_path):
    import ctypes as C
    import shutil
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "transims.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n",'
                   'sizeof(sim_config),sizeof(sim_params),sizeof(sim_network),'
                   'sizeof(sim_vehicles),sizeof(sim_stats_t),sizeof(sim_tiling),'
                   'sizeof(sim_kernel_time));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"),
                           str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(t) for t in (sim.sim_config, sim.sim_params,
                                  sim.sim_network, sim.sim_vehicles,
                                  sim.sim_stats_t, sim.sim_tiling,
                                  sim.sim_kernel_time)]
    assert got == want
