"""Writes the full-length oracle references of the two long single-lattice
workloads into tests/golden/.  It calls only the CPU oracle (oracle/) and the
input recipes (paper_2508_16639_amd/workloads.py, which holds no method
arithmetic); nothing here comes from the HIP path.

For each workload the oracle's parallel-schedule reference (O2) runs the
whole job from the method's own initial lattice and records the species
counts before the first MCS and after every MCS, as the paper's Overall ESCG
Loop records densities every MCS:

  rpsls_L3200_1000mcs.txt  RPSLS (S = 5, i beats i+1 and i+3), L = 3200,
                           M = 1e-5 (eps = 51.2), sigma = mu = 1, seed 1,
                           1000 MCS: 1001 rows of 6 counts
  rps_L512_10000mcs.txt    RPS (S = 3), L = 512, M = 1e-4 (eps = 13.1072),
                           sigma = mu = 1, seed 1, 10000 MCS: 10001 rows of
                           4 counts

Each file starts with '#' header lines (the workload, the generator, the
SHA-256 of the final lattice bytes, row-major uint8[L*L]), then one line per
count row, counts separated by single spaces.

Usage:  python tests/golden/make_full_length.py [rpsls_L3200 | rps_L512]...
(no argument: both; about 5 and 2 minutes of one CPU core).
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2508_16639_amd.workloads import RPS512, RPSLS3200  # noqa: E402

OUT = {"rpsls_L3200": (RPSLS3200, "rpsls_L3200_1000mcs.txt"),
       "rps_L512": (RPS512, "rps_L512_10000mcs.txt")}


def write(name: str) -> str:
    w, fname = OUT[name]
    job = O.Job(w.L, w.S, O.circulant_matrix(w.S, w.K), w.ex, w.sel, w.rep,
                seed=w.seed, replica=w.replica)
    t0 = time.time()
    g = job.init()
    c = O.o2_run(job, g, 0, w.mcs)
    sha = hashlib.sha256(g.tobytes()).hexdigest()
    path = os.path.join(HERE, fname)
    with open(path, "w") as f:
        f.write(f"# workload {w.name}: L={w.L} S={w.S} K={list(w.K)} "
                f"ex={w.ex!r} sel={w.sel!r} rep={w.rep!r} seed={w.seed} "
                f"replica={w.replica} mcs={w.mcs}\n")
        f.write(f"# generator: oracle O2 (Philox4x32-{job.rounds}), "
                f"tests/golden/make_full_length.py\n")
        f.write(f"# final_lattice_sha256 {sha}\n")
        f.write(f"# rows {c.shape[0]} cols {c.shape[1]}: counts of "
                f"v = 0..S before the first MCS and after each MCS\n")
        for row in c:
            f.write(" ".join(str(int(v)) for v in row) + "\n")
    print(f"{name}: {c.shape[0]} rows, sha256 {sha}, "
          f"{time.time() - t0:.1f} s -> {path}", flush=True)
    return path


def read(fname: str):
    """(counts uint32[rows, S+1], final-lattice SHA-256 hex, header dict)."""
    sha, rounds = None, None
    with open(os.path.join(HERE, fname)) as f:
        for line in f:
            if not line.startswith("#"):
                break
            if line.startswith("# final_lattice_sha256"):
                sha = line.split()[2]
            if line.startswith("# generator: oracle O2 (Philox4x32-"):
                rounds = int(line.split("Philox4x32-")[1].split(")")[0])
    c = np.loadtxt(os.path.join(HERE, fname), dtype=np.uint32, comments="#",
                   ndmin=2)
    return c, sha, {"rounds": rounds}


if __name__ == "__main__":
    names = sys.argv[1:] or list(OUT)
    for n in names:
        write(n)
