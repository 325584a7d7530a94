"""Builds the HIP library ``libescg.so`` for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(PKG, "libescg.so")
SOURCES = [os.path.join(CSRC, "escg.hip")]
HEADERS = [os.path.join(CSRC, "escg_device.hpp"),
           os.path.join(CSRC, "escg_quad.hpp"),
           os.path.join(CSRC, "escg_lds.hpp"),
           os.path.join(CSRC, "escg_tile.hpp"),
           os.path.join(INCLUDE, "escg.h")]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-result",
    # no packed fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; cannot build the ESCG library")
    return exe



def build(verbose: bool = False) -> str:
    """Compiles libescg.so (always; no staleness shortcut)."""
    tmp = LIB_PATH + f".tmp{os.getpid()}"
    cmd = [hipcc(), *HIPCC_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", *SOURCES,
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
