#!/usr/bin/env python3
"""Benchmark of the ESCG Monte Carlo hot path on one MI355X.

Headline (one "step" = the whole hot path over one synthetic input): RPSLS
(S = 5, i beats i+1 and i+3 mod 5) on an L = 3200 periodic lattice, mobility
M = 1e-5 (eps = M L^2 / 2 = 51.2, sel = rep = 1), seed 1: initialise the
lattice on the device, then 1,000 MCS with species counts after every MCS.
value = site-updates/s = L^2 * 1000 * steps / wall time of the timed steps.

Also reported on the same GPU:
  batch      4,096 RPS replicas (L uniform over {64,128,192,256}, log10 M
             uniform on [-6,-3], stop at first extinction or 20 L MCS) in one
             persistent launch, in replica-jobs/s, beside plain one-job-at-a-
             time launches on a sample of the same table;
  serving    the continuous-batching job server on a Poisson request stream
             (see paper_2508_16639_amd/serve.py), jobs/s with p50/p99 latency
             beside plain one-at-a-time serving;
  roofline   algorithmic HBM bytes (2 B per site-update: every site read and
             written once per MCS) of the dominant kernel divided by its
             average launch duration from HIP events on the launch stream;
             HBM traffic from rocprofv3 counters when the recorded profile
             matches the current kernel source;
  cpu_baseline  the oracle (same schedule, single thread) on a bounded
             sample of the headline workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
VALU_PEAK_TLANEOPS = 39.32     # 256 CU * 4 SIMD * 16 lanes * 2.4 GHz, int32 VALU
BYTES_PER_SU = 2.0             # read + write of one uint8 site per update


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2508_16639_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_profile(name: str):
    """Counter-derived figures recorded under profiles/ for the current
    kernel source, else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec


def headline(args, torch, escg, w, p):
    N = w.L * w.L
    lat = torch.empty(N, dtype=torch.uint8, device="cuda")
    cnt = torch.empty((w.mcs + 1) * (w.S + 1), dtype=torch.int32,
                      device="cuda")
    events = []

    def step(timed):
        escg.init(p, lat)
        if timed:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
        escg.step_mcs(p, lat, 0, w.mcs, cnt)
        if timed:
            e1.record()
            events.append((e0, e1))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    escg.async_status()
    c = cnt.cpu().numpy().reshape(w.mcs + 1, w.S + 1)
    assert (c.sum(1) == N).all(), "species counts do not sum to L^2"
    kern_ms = sum(a.elapsed_time(b) for a, b in events) / len(events)
    su = float(N) * w.mcs
    return {
        "value": su * args.steps / wall,
        "ms_per_step": wall / args.steps * 1e3,
        "kernel_ms": kern_ms,
        "su_per_launch": su,
        "final_counts": c[-1].tolist(),
    }


def batch(args, torch, escg, workloads):
    tab = workloads.batch_replicas()
    n = len(tab)
    dom = escg.circulant_dom(3, [1])
    params, offs, off = [], [], 0
    for r in range(n):
        L = int(tab.L[r])
        params.append(escg.Params(L=L, S=3, dom=dom, ex=float(tab.ex[r]),
                                  seed=tab.seed, replica=r))
        offs.append(off)
        off += L * L
    buf = torch.empty(off, dtype=torch.uint8, device="cuda")
    res = torch.empty(n * escg.BATCH_RESULT_WORDS, dtype=torch.int32,
                      device="cuda")
    reps = max(1, min(3, args.steps))
    escg.batch_run(params, offs, buf, tab.max_mcs,
                   escg.STOP_FIRST_EXTINCTION, True, res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        escg.batch_run(params, offs, buf, tab.max_mcs,
                       escg.STOP_FIRST_EXTINCTION, True, res)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    r = res.cpu().numpy().reshape(n, escg.BATCH_RESULT_WORDS)
    su = float((tab.L.astype(float) ** 2 * r[:, 1]).sum())
    # plain: one job at a time (init + run until extinction + sync), on the
    # first `k` replicas of the same table
    k = 32
    one = torch.empty(256 * 256, dtype=torch.uint8, device="cuda")
    out = torch.empty(6, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    su_plain = 0.0
    for i in range(k):
        q = params[i]
        escg.init(q, one)
        escg.run_until_extinction(q, one, 0, int(tab.max_mcs[i]),
                                  escg.STOP_FIRST_EXTINCTION, out)
        torch.cuda.synchronize()
        su_plain += float(q.L) ** 2 * int(out[1].item())
    plain_wall = time.perf_counter() - t0
    return {
        "workload": "4096 RPS replicas, L in {64,128,192,256}, "
                    "M log-uniform [1e-6,1e-3], first extinction or 20 L MCS",
        "jobs_per_s": n / wall,
        "site_updates_per_s": su / wall,
        "seconds": wall,
        "extinct_fraction": float(r[:, 0].mean()),
        "plain_jobs_per_s": k / plain_wall,
        "plain_site_updates_per_s": su_plain / plain_wall,
        "plain_sample": f"first {k} replicas, one at a time on one stream",
        "speedup_vs_plain": (n / wall) / (k / plain_wall),
    }


def serving(args, torch, escg, workloads):
    try:
        from paper_2508_16639_amd import serve
    except ImportError:
        return None
    return serve.bench_serving(torch, escg, workloads)


def host_cpu() -> str:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model or 'unknown CPU'}, {os.cpu_count()} logical CPUs visible"


def cpu_baseline(w):
    import oracle as O
    n = 50
    job = O.Job(w.L, w.S, O.circulant_matrix(w.S, w.K), w.ex, w.sel, w.rep,
                seed=w.seed, replica=w.replica)
    t0 = time.perf_counter()
    g = job.init()
    c = O.o2_run(job, g, 0, n)
    dt = time.perf_counter() - t0
    assert (c.sum(1) == w.L * w.L).all()
    return {"value": float(w.L) ** 2 * n / dt, "unit": "site-updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"oracle (same block schedule, plain C, one thread): "
                      f"L={w.L} RPSLS init + {n} of the {w.mcs} MCS with "
                      f"per-MCS counts, {dt:.1f} s; host {host_cpu()}"}


def _o2_replica(args):
    import oracle as O
    L, S, K, ex, seed, replica, n = args
    job = O.Job(L, S, O.circulant_matrix(S, K), ex, seed=seed,
                replica=replica)
    g = job.init()
    O.o2_run(job, g, 0, n, want_counts=False)
    return L * L * n


def cpu_context(w):
    """Further CPU figures beside the baseline: the paper-style random-
    sequential oracle (O1) on one thread, and the block-schedule oracle on
    every core with one replica per process (independent replicas are the
    CPU's natural parallelism)."""
    import multiprocessing as mp
    import oracle as O
    job = O.Job(w.L, w.S, O.circulant_matrix(w.S, w.K), w.ex, w.sel, w.rep,
                seed=w.seed, replica=w.replica)
    g = job.init()
    n1 = 10
    t0 = time.perf_counter()
    O.o1_run(job, g, 0, n1, want_counts=False)
    d1 = time.perf_counter() - t0
    cores = max(1, min(16, os.cpu_count() or 1))
    L, n = 800, 200  # per replica: 1.28e8 site-updates
    tasks = [(L, w.S, list(w.K), w.ex, w.seed, r, n) for r in range(cores)]
    t0 = time.perf_counter()
    with mp.Pool(cores) as pool:
        su = sum(pool.map(_o2_replica, tasks))
    dall = time.perf_counter() - t0
    return {"o1_one_thread": {"value": float(w.L) ** 2 * n1 / d1,
                              "unit": "site-updates/s",
                              "sample": f"L={w.L} RPSLS, {n1} MCS, "
                                        f"{d1:.1f} s"},
            "o2_all_cores": {"value": su / dall, "unit": "site-updates/s",
                             "cores": cores,
                             "sample": f"{cores} replicas of L={L} RPSLS "
                                       f"x {n} MCS, one per process, "
                                       f"{dall:.1f} s"},
            "host": host_cpu()}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--skip-extras", action="store_true",
                    help="headline only (no batch, serving, cpu baseline)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="only run device-to-device copies of this many MiB "
                         "(reference for rocprofv3 byte counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU "
              "path (independent replicas and jobs would shard by seed and "
              "replica id with no communication); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2508_16639_amd import escg, workloads
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": args.steps}))
        return
    escg.lib()
    w = workloads.RPSLS3200

    from paper_2508_16639_amd import autotune
    p = escg.Params(L=w.L, S=w.S, dom=escg.circulant_dom(w.S, w.K), ex=w.ex,
                    sel=w.sel, rep=w.rep, seed=w.seed, replica=w.replica)
    tuned = autotune.apply(torch, p, "persistent")
    shape = tuned.tile if tuned is not p else None
    p = tuned
    plan = escg.tile_plan(p, True)
    log(f"[bench] headline {w.name}: warmup {args.warmup}, steps {args.steps}, "
        f"tile plan {plan} (autotuned: {shape is not None}, "
        f"device {autotune.device_key(torch)})")
    h = headline(args, torch, escg, w, p)
    log(f"[bench] headline {h['value']:.4e} site-updates/s, "
        f"{h['ms_per_step']:.2f} ms/step, kernel {h['kernel_ms']:.2f} ms")
    achieved = BYTES_PER_SU * h["su_per_launch"] / (h["kernel_ms"] * 1e-3) / 1e9
    prof = recorded_profile("counters_rpsls_L3200.json")
    traffic = prof.get("hbm_bytes_per_launch") if prof else None
    alu = None
    if prof and prof.get("valu_lane_ops_per_launch"):
        # wave64 VALU instructions x 64 lanes per kernel second (every
        # integer VALU instruction the kernel uses issues at full rate,
        # v_mad_u64_u32 included: tests/microbench/valu_rates.hip)
        a = prof["valu_lane_ops_per_launch"] / (h["kernel_ms"] * 1e-3) / 1e12
        alu = {"bound": "alu", "achieved": a, "peak": VALU_PEAK_TLANEOPS,
               "unit": "T lane-instr/s", "frac": a / VALU_PEAK_TLANEOPS,
               "note": "SQ_INSTS_VALU x 64 per launch (profiles/counters_"
                       "rpsls_L3200.json) over the live kernel time; peak "
                       "256 CU x 4 SIMD x 16 lanes x 2.4 GHz"}
    out = {
        "metric": "site-updates/s at L=3200 (RPSLS, 1000 MCS, counts every "
                  "MCS) + replica-jobs/s with p50/p99 latency vs plain",
        "value": h["value"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "rpsls_L3200_M1e-5_1000mcs", "L": w.L,
                   "S": w.S, "K": list(w.K), "eps": w.ex, "mcs": w.mcs,
                   "seed": w.seed, "counts_every_mcs": True,
                   "parallelism": "single GPU, persistent tiled kernel",
                   "tile_TH_TW_threads": list(plan) if plan else None,
                   "tile_shape_autotuned": shape is not None},
        "roofline": {"bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "tiled_persistent_kernel",
                     "kernel_ms": h["kernel_ms"],
                     "algorithmic_bytes_per_launch":
                         BYTES_PER_SU * h["su_per_launch"]},
        "alu": alu,
        "context": {"paper_cuda_ms_L3200_rtx_a2000_su_per_s": 2.45e8,
                    "note": "the paper's CUDA --maxStep run at L=3200 (RPS, "
                            "1e5 MCS, unstated mobility) took 4173.5 s; "
                            "another machine and workload, context only"},
    }
    if not args.skip_extras:
        log("[bench] batch (4096 replicas)")
        out["batch"] = batch(args, torch, escg, workloads)
        log(f"[bench] batch {out['batch']['jobs_per_s']:.1f} jobs/s")
        log("[bench] serving")
        out["serving"] = serving(args, torch, escg, workloads)
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w)
        log("[bench] cpu context (O1, all-core O2)")
        out["cpu_context"] = cpu_context(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
