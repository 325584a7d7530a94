"""Host emulation of the device kernels' lattice logic against the oracle.

The device headers (quad update, whole-lattice pass, tile load / walk /
passes / halo publish and gather / counts) are compiled for the host with
g++ and a small shim of the HIP built-ins they use (tests/emu/hip), the
threads of a workgroup run one after another (the passes touch disjoint
blocks, so that order gives the parallel result), and the lattices and
counts are compared byte for byte with the oracle (oracle/escg_oracle.c,
O2).  Two textual substitutions make the headers host-compilable: the two
inline-asm helpers become their C equivalents, and the count's wave sum
becomes a per-thread add (a thread's own value is its wave's sum when the
threads run one at a time).  Cross-lane steps of the counts are recomputed
in the test programs.  No GPU is needed.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_16639_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")
ORACLE_C = os.path.join(ROOT, "oracle", "escg_oracle.c")

pytestmark = pytest.mark.skipif(
    shutil.which("g++") is None or shutil.which("gcc") is None,
    reason="needs gcc and g++")


def _host_headers(dst: str) -> None:
    for name in os.listdir(CSRC):
        if name.endswith(".hpp"):
            shutil.copy(os.path.join(CSRC, name), dst)
    p = os.path.join(dst, "escg_device.hpp")
    s = open(p).read()
    a = s.index('    uint32_t r;\n    asm("v_bitop3_b32')
    b = s.index("    return r;\n", a) + len("    return r;\n")
    s = s[:a] + "    return a ^ b ^ k;\n" + s[b:]
    a = s.index('    uint32_t r;\n    asm volatile("v_mov_b32')
    b = s.index("    return r;\n", a) + len("    return r;\n")
    s = s[:a] + "    return k;\n" + s[b:]
    open(p, "w").write(s)
    p = os.path.join(dst, "escg_tile.hpp")
    s = open(p).read()
    assert "(threadIdx.x & 63u) == 0 && tot" in s
    s = s.replace("(threadIdx.x & 63u) == 0 && tot", "tot")
    open(p, "w").write(s)


@pytest.fixture(scope="module")
def emu_dir(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("emu"))
    src = os.path.join(d, "src")
    os.makedirs(src)
    _host_headers(src)
    orc = os.path.join(d, "orc.o")
    subprocess.check_call(["gcc", "-O1", "-c", ORACLE_C, "-o", orc])
    return d


@pytest.mark.parametrize("prog,expect", [("emu_lds", "cases ok"),
                                         ("emu_tile", "tiled cases ok")])
def test_device_logic_matches_oracle(emu_dir, prog, expect):
    exe = os.path.join(emu_dir, prog)
    subprocess.check_call(
        ["g++", "-O1", "-std=c++17", f"-I{EMU}", f"-I{emu_dir}/src",
         os.path.join(EMU, prog + ".cpp"), os.path.join(emu_dir, "orc.o"),
         "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    last = r.stdout.strip().splitlines()[-1]
    assert r.returncode == 0, r.stdout[-2000:]
    n_ok, n = last.split()[0].split("/")
    assert expect in last and n_ok == n and int(n) > 0, last
