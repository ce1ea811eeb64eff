"""Builds libtransims.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtransims.so")
SOURCES = ["csrc/transims.cpp", "csrc/tiler.cpp", "csrc/step.hip",
           "csrc/front_back.hip", "csrc/ring_stats.hip", "csrc/scratch.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> str:
    """Compiles every source into paper_cs_0105004_amd/libtransims.so."""
    objs = []
    tmpdir = os.path.join(HERE, "_build")
    os.makedirs(tmpdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall",
              "-I" + os.path.join(ROOT, "include")]
    for src in SOURCES:
        path = os.path.join(HERE, src)
        obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
        cmd = [hipcc()] + common
        if src.endswith(".hip"):
            cmd += ["-x", "hip", "--offload-arch=" + ARCH,
                    # keep the compiler from emitting packed fp32 arithmetic
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        cmd += ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
