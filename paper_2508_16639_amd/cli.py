"""Command-line simulation driver with the paper's run options.

    python -m paper_2508_16639_amd.cli --length 400 --mcs 20000 \\
        --mobility 3e-5 --species 3 --printFrequency 200 --save out/

The flags mirror the paper's program (Sec. "Single Threaded ESCG in C++",
table of command-line parameters; CUDA section, additional flags):
--length/--height (square lattices only), --mcs (MCS limit), --neighbourhood
(4 = von Neumann, 8 = Moore), --printFrequency, --mobility
(eps = M * L^2 / 2, escg_eps_from_mobility), --species, --flux (periodic
boundaries only), --empty (initial empty-site probability), --save,
--dominance (import a dominance CSV; it sets the species count, and
entries strictly between 0 and 1 are win probabilities), --resume
(continue a saved run).  --numRandoms and --maxStep are accepted and have no
effect: random numbers are drawn inside the kernels, and a single launch
already runs many MCS.

Every MCS runs on the GPU through the C ABI (escg.step_mcs with per-MCS
counts); this module only parses options, moves files and prints.  The run
stops at the MCS limit or, as the paper's loop does, at monoculture (at most
one species left); the stop is exact: a chunk that passes the stop is
re-run from its saved start up to the stopping MCS.

Saved run directory: params.csv, dominance.csv, grid.csv (lattice and MCS
done, written every --saveFrequency MCS and at the end) and densities.csv
(every MCS).  Because every draw is keyed by (seed, replica, MCS, pass,
site), a resumed run continues byte for byte as if it had never stopped.
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from typing import List, Optional

import numpy as np

from . import escg_io


def _flag(v: str) -> bool:
    t = str(v).strip().lower()
    if t in ("1", "true", "yes", "on"):
        return True
    if t in ("0", "false", "no", "off"):
        return False
    raise argparse.ArgumentTypeError(f"expected true/false, got {v!r}")


def build_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser(
        prog="python -m paper_2508_16639_amd.cli",
        description="ESCG lattice simulation on the GPU (MI355X).")
    ap.add_argument("--length", type=int, default=200)
    ap.add_argument("--height", type=int, default=None,
                    help="must equal --length (square lattices)")
    ap.add_argument("--mcs", type=int, default=100000,
                    help="MCS limit (total, counting resumed MCS)")
    ap.add_argument("--neighbourhood", type=int, default=4, choices=(4, 8))
    ap.add_argument("--printFrequency", type=int, default=200)
    ap.add_argument("--mobility", type=float, default=3e-5)
    ap.add_argument("--species", type=int, default=3)
    ap.add_argument("--flux", type=_flag, default=True,
                    help="periodic (wrap) boundaries; only true is supported")
    ap.add_argument("--empty", type=float, default=None,
                    help="initial empty-site probability; other sites take "
                         "species 1..S uniformly (default: every state "
                         "0..S equally likely, the library's escg_init)")
    ap.add_argument("--save", default=None,
                    help="output directory ('true' = a name built from the "
                         "run's parameters)")
    ap.add_argument("--saveFrequency", type=int, default=0,
                    help="MCS between grid snapshots (0 = only at the end)")
    ap.add_argument("--dominance", default=None,
                    help="dominance CSV to import ('true' = dominance.csv)")
    ap.add_argument("--offsets", default=None,
                    help="circulant dominance offsets K, comma separated "
                         "(default: 1 for S = 3, 1,3 for S = 5, else 1)")
    ap.add_argument("--resume", default=None,
                    help="saved run directory to continue")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--replica", type=int, default=0)
    ap.add_argument("--selection", type=float, default=1.0)
    ap.add_argument("--reproduction", type=float, default=1.0)
    ap.add_argument("--numRandoms", type=int, default=None,
                    help="accepted for compatibility; no effect")
    ap.add_argument("--maxStep", type=_flag, default=False,
                    help="accepted for compatibility; no effect")
    ap.add_argument("--quiet", action="store_true")
    return ap


def _default_offsets(S: int) -> List[int]:
    return [1, 3] if S == 5 else [1]


def _monoculture(row: np.ndarray) -> bool:
    return int((np.asarray(row[1:]) > 0).sum()) <= 1


class Run:
    """The state of one simulation: parameters, device lattice, MCS done."""

    def __init__(self, args, torch, escg):
        self.args, self.torch, self.escg = args, torch, escg
        resume = args.resume
        if resume:
            prm = escg_io.read_params_csv(os.path.join(resume, "params.csv"))
            D, P = escg_io.read_dominance_probabilities_csv(
                os.path.join(resume, "dominance.csv"))
            g, L, done = escg_io.read_grid_csv(os.path.join(resume,
                                                            "grid.csv"))
            self.L, self.S = L, D.shape[0]
            self.moore = int(prm.get("neighbourhood", "4")) == 8
            self.mobility = float(prm["mobility"])
            self.seed = int(prm["seed"])
            self.replica = int(prm["replica"])
            self.sel = float(prm["selection"])
            self.rep = float(prm["reproduction"])
            self.D, self.P = D, P
            self.done = done
            self.lattice0 = g
        else:
            if args.height is not None and args.height != args.length:
                raise SystemExit("only square lattices: --height must equal "
                                 "--length")
            if not args.flux:
                raise SystemExit("only periodic boundaries (--flux true)")
            self.L = args.length
            if args.dominance:
                path = ("dominance.csv" if str(args.dominance).lower() ==
                        "true" else args.dominance)
                self.D, self.P = escg_io.read_dominance_probabilities_csv(
                    path)
                self.S = self.D.shape[0]
            else:
                self.S = args.species
                K = ([int(k) for k in args.offsets.split(",")]
                     if args.offsets else _default_offsets(self.S))
                dom = escg.circulant_dom(self.S, K)
                self.D = np.array([[(dom[a] >> b) & 1
                                    for b in range(1, self.S + 1)]
                                   for a in range(1, self.S + 1)], np.uint8)
                self.P = None
            self.moore = args.neighbourhood == 8
            self.mobility = args.mobility
            self.seed, self.replica = args.seed, args.replica
            self.sel, self.rep = args.selection, args.reproduction
            self.done = 0
            self.lattice0 = None
        self.N = self.L * self.L
        eps = escg.eps_from_mobility(self.mobility, self.L)
        self.p = escg.Params(L=self.L, S=self.S,
                             dom=escg.dom_from_matrix(self.D), ex=eps,
                             sel=self.sel, rep=self.rep, seed=self.seed,
                             replica=self.replica, moore=self.moore,
                             prob=self.P)
        self.lat = torch.empty(self.N, dtype=torch.uint8, device="cuda")
        if self.lattice0 is not None:
            if int(self.lattice0.max()) > self.S:
                raise SystemExit("saved grid holds values above S")
            self.lat.copy_(torch.from_numpy(self.lattice0))
        elif args.empty is not None:
            if not 0.0 <= args.empty <= 1.0:
                raise SystemExit("--empty must be in [0, 1]")
            rng = np.random.default_rng([self.seed, self.replica])
            g = rng.integers(1, self.S + 1, size=self.N, dtype=np.uint8)
            g[rng.random(self.N) < args.empty] = 0
            self.lat.copy_(torch.from_numpy(g))
        else:
            escg.init(self.p, self.lat)

    def params_record(self):
        return {"length": self.L, "height": self.L, "species": self.S,
                "mobility": repr(self.mobility), "seed": self.seed,
                "replica": self.replica, "selection": repr(self.sel),
                "reproduction": repr(self.rep),
                "neighbourhood": 8 if self.moore else 4, "flux": "true"}

    def host_lattice(self) -> np.ndarray:
        self.torch.cuda.synchronize()
        return self.lat.cpu().numpy()

    def advance(self, n: int):
        """n MCS from self.done with counts; returns the count rows
        (rows 1..k after each MCS) and whether monoculture stopped it."""
        torch, escg = self.torch, self.escg
        start = self.lat.clone()
        cnt = torch.empty((n + 1) * (self.S + 1), dtype=torch.int32,
                          device="cuda")
        escg.step_mcs(self.p, self.lat, self.done, n, cnt)
        # a persistent launch that gave up a neighbour wait leaves an
        # invalid lattice: raise (EscgError) before anything is written
        escg.async_status()
        rows = cnt.cpu().numpy().view(np.uint32).reshape(n + 1, self.S + 1)
        for k in range(1, n + 1):
            if _monoculture(rows[k]):
                if k < n:  # re-run exactly k MCS from the chunk's start
                    self.lat.copy_(start)
                    escg.step_mcs(self.p, self.lat, self.done, k, None)
                    escg.async_status()
                self.done += k
                return rows[1:k + 1], True
        self.done += n
        return rows[1:], False


def main(argv: Optional[List[str]] = None) -> int:
    args = build_parser().parse_args(argv)
    import torch
    from . import escg
    escg.lib()
    run = Run(args, torch, escg)
    escg.async_status()  # start from a clean device error record
    out = None
    if args.save or args.resume:
        out = args.resume if (args.resume and not args.save) else args.save
        if out and str(out).lower() == "true":
            out = escg_io.run_dir_name(run.L, run.S, run.mobility,
                                       "moore" if run.moore else "vn")
        os.makedirs(out, exist_ok=True)
        escg_io.write_params_csv(os.path.join(out, "params.csv"),
                                 run.params_record())
        escg_io.write_dominance_csv(os.path.join(out, "dominance.csv"), run.D,
                                    run.P)
    dens = os.path.join(out, "densities.csv") if out else None
    c0 = torch.empty(run.S + 1, dtype=torch.int32, device="cuda")
    escg.densities(run.p, run.lat, c0)
    c0 = c0.cpu().numpy().view(np.uint32)
    if dens and run.done == 0:
        if os.path.exists(dens):
            os.remove(dens)
        escg_io.append_densities_csv(dens, c0[None, :], 0, run.N)
    pf = max(1, args.printFrequency)
    sf = args.saveFrequency
    t0 = time.perf_counter()
    stopped = _monoculture(c0)  # the paper's loop tests before each MCS
    while run.done < args.mcs and not stopped:
        n = min(pf, args.mcs - run.done)
        if sf > 0:
            n = min(n, sf - run.done % sf)
        first = run.done + 1
        rows, stopped = run.advance(n)
        if dens:
            escg_io.append_densities_csv(dens, rows, first, run.N)
        if not args.quiet and (run.done % pf == 0 or stopped or
                               run.done == args.mcs):
            d = rows[-1] / run.N
            print(f"MCS {run.done}: " + " ".join(
                f"{v:.4f}" for v in d), flush=True)
        if out and sf > 0 and run.done % sf == 0:
            escg_io.write_grid_csv(os.path.join(out, "grid.csv"),
                                   run.host_lattice(), run.L, run.done)
    wall = time.perf_counter() - t0
    if out:
        escg_io.write_grid_csv(os.path.join(out, "grid.csv"),
                               run.host_lattice(), run.L, run.done)
    if not args.quiet:
        why = "monoculture" if stopped else "MCS limit"
        print(f"stopped at MCS {run.done} ({why}); {wall:.2f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
