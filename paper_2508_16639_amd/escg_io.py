"""Host-side files of a simulation run: the dominance matrix, lattice
snapshots, run parameters and the per-MCS density record, all as CSV.

Formats follow the paper's program (Sec. "Single Threaded ESCG in C++":
dominance import; CUDA section: save / resume):
  * dominance CSV: S rows of S comma-separated entries, row i = species
    i+1, column j = species j+1, 1 = row species beats column species
    (the paper's flat matrix layout of Algorithm "Dominance Check"); the
    number of rows sets S; entries strictly between 0 and 1 are win
    probabilities (probabilistic dominance);
  * grid CSV: one line per lattice row of comma-separated site values
    (0 = empty, 1..S species), then one line with the number of MCS done;
  * params CSV: `name,value` lines;
  * densities CSV: header `mcs,empty,species_1,...,species_S`, one line per
    recorded MCS with each state's fraction of the N = L*L sites.
Only numpy is used here; no simulation arithmetic.
"""
from __future__ import annotations

import csv
import os
from typing import Dict, Tuple

import numpy as np


def read_dominance_csv(path: str) -> np.ndarray:
    """S x S uint8 matrix (0/1) from a dominance CSV; raises ValueError on a
    non-square matrix, entries other than 0/1 or S outside 1..31."""
    D, P = read_dominance_probabilities_csv(path)
    if P is not None:
        raise ValueError(f"{path}: entries must be 0 or 1")
    return D


def read_dominance_probabilities_csv(path: str):
    """(D, P) from a dominance CSV whose entries are win probabilities in
    [0, 1] (the probabilistic interactions of the Park, Chen and Szolnoki
    replication): D = (entry > 0) as uint8, P the float matrix, or None when
    every entry is 0 or 1 (a deterministic matrix)."""
    rows = []
    with open(path, newline="") as f:
        for line in csv.reader(f):
            cells = [c.strip() for c in line if c.strip() != ""]
            if cells:
                rows.append([float(c) for c in cells])
    S = len(rows)
    if not 1 <= S <= 31 or any(len(r) != S for r in rows):
        raise ValueError(f"{path}: expected a square matrix with 1..31 rows")
    P = np.asarray(rows, dtype=np.float64)
    if not ((P >= 0.0) & (P <= 1.0)).all():
        raise ValueError(f"{path}: entries must lie in [0, 1]")
    D = (P > 0.0).astype(np.uint8)
    return D, (None if np.isin(P, (0.0, 1.0)).all() else P)


def write_dominance_csv(path: str, D: np.ndarray, P=None) -> None:
    """Writes D (0/1), or the probabilities P where given (exact reprs)."""
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        if P is None:
            for row in np.asarray(D, dtype=np.uint8):
                w.writerow([int(v) for v in row])
        else:
            for row in np.asarray(P, dtype=np.float64):
                w.writerow([repr(float(v)) for v in row])


def write_grid_csv(path: str, lattice: np.ndarray, L: int, mcs: int) -> None:
    g = np.asarray(lattice, dtype=np.uint8).reshape(L, L)
    with open(path, "w") as f:
        for row in g:
            f.write(",".join(str(int(v)) for v in row))
            f.write("\n")
        f.write(f"{int(mcs)}\n")


def read_grid_csv(path: str) -> Tuple[np.ndarray, int, int]:
    """(flat uint8 lattice, L, MCS done) from a grid CSV."""
    with open(path) as f:
        lines = [ln.strip() for ln in f if ln.strip()]
    if len(lines) < 2:
        raise ValueError(f"{path}: need lattice rows and a final MCS line")
    mcs = int(lines[-1])
    rows = [[int(c) for c in ln.split(",")] for ln in lines[:-1]]
    L = len(rows)
    if any(len(r) != L for r in rows):
        raise ValueError(f"{path}: the lattice must be square")
    g = np.asarray(rows, dtype=np.int64)
    if g.min() < 0 or g.max() > 255:
        raise ValueError(f"{path}: site values out of range")
    return g.astype(np.uint8).reshape(-1), L, mcs


def write_params_csv(path: str, params: Dict[str, object]) -> None:
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        for k, v in params.items():
            w.writerow([k, v])


def read_params_csv(path: str) -> Dict[str, str]:
    with open(path, newline="") as f:
        return {r[0]: r[1] for r in csv.reader(f) if len(r) >= 2}


def densities_header(S: int) -> str:
    return ",".join(["mcs", "empty"] + [f"species_{s}" for s in range(1, S + 1)])


def append_densities_csv(path: str, counts: np.ndarray, first_mcs: int,
                         N: int) -> None:
    """Appends rows (first_mcs + i, counts[i] / N) for each row i of the
    (rows, S+1) count array; writes the header if the file is new."""
    counts = np.asarray(counts, dtype=np.float64).reshape(counts.shape[0], -1)
    new = not os.path.exists(path)
    with open(path, "a") as f:
        if new:
            f.write(densities_header(counts.shape[1] - 1) + "\n")
        for i, row in enumerate(counts):
            f.write(",".join([str(first_mcs + i)] +
                             [repr(float(v) / N) for v in row]) + "\n")


def read_densities_csv(path: str) -> Tuple[np.ndarray, np.ndarray]:
    """(mcs indices, densities (rows, S+1)) from a densities CSV."""
    with open(path) as f:
        lines = [ln.strip() for ln in f if ln.strip()]
    body = [[float(c) for c in ln.split(",")] for ln in lines[1:]]
    a = np.asarray(body, dtype=np.float64).reshape(len(body), -1)
    return a[:, 0].astype(np.int64), a[:, 1:]


def run_dir_name(L: int, S: int, mobility: float, neighbourhood: str = "vn",
                 boundary: str = "periodic") -> str:
    """Output directory named by the run's key parameters (lattice size,
    neighbourhood, mobility, boundary, species count), as the paper's
    program does."""
    return f"L{L}x{L}_{neighbourhood}_M{mobility:g}_{boundary}_S{S}"

