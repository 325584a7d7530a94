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

import numpy as np

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
    from paper_2508_16639_amd import autotune
    sides = tuple(sorted(set(int(x) for x in tab.L)))
    tuned = autotune.lookup(torch, "batch", sides, 3)
    launch = {"autotuned": tuned is not None,
              **autotune.launch_choice(tuned)}
    if tuned:
        params[0] = params[0].with_launch(**autotune.launch_choice(tuned))
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
    # plain: one job at a time (init + run until extinction + sync), on a
    # seeded random sample of the same table
    k = min(n, 128)
    pick = np.random.default_rng(12345).choice(n, size=k, replace=False)
    one = torch.empty(256 * 256, dtype=torch.uint8, device="cuda")
    out = torch.empty(6, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    times, su_plain = [], 0.0
    for i in pick:
        q = params[int(i)]
        t1 = time.perf_counter()
        escg.init(q, one)
        escg.run_until_extinction(q, one, 0, int(tab.max_mcs[i]),
                                  escg.STOP_FIRST_EXTINCTION, out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        su_plain += float(q.L) ** 2 * int(out[1].item())
    times = np.asarray(times)
    mean, se = times.mean(), times.std(ddof=1) / np.sqrt(k)
    plain_jps = 1.0 / mean
    lo, hi = 1.0 / (mean + 1.96 * se), 1.0 / max(mean - 1.96 * se, 1e-12)
    return {
        "workload": "4096 RPS replicas, L in {64,128,192,256}, "
                    "M log-uniform [1e-6,1e-3], first extinction or 20 L MCS",
        "jobs_per_s": n / wall,
        "site_updates_per_s": su / wall,
        "su_per_job": su / n,
        "seconds": wall,
        "extinct_fraction": float(r[:, 0].mean()),
        "launch": launch,
        "plain_jobs_per_s": plain_jps,
        "plain_jobs_per_s_95ci": [lo, hi],
        "plain_site_updates_per_s": su_plain / times.sum(),
        "plain_sample": f"{k} replicas drawn at random (seed 12345) from the "
                        f"table, one at a time on one stream (init, run "
                        f"until extinction, synchronise); 95 % interval "
                        f"from the sample's per-job times",
        "speedup_vs_plain": (n / wall) / plain_jps,
        "speedup_vs_plain_95ci": [(n / wall) / hi, (n / wall) / lo],
    }


def serving(args, torch, escg, workloads):
    from paper_2508_16639_amd import serve
    return serve.bench_serving(torch, escg, workloads)


def rps512(args, torch, escg, workloads):
    """The L = 512 RPS workload (10,000 MCS, counts every MCS): init and
    the whole run per repetition, on the route the library picks, with the
    autotuned tile shape where the cache has one."""
    from paper_2508_16639_amd import autotune
    w = workloads.RPS512
    p = escg.Params(L=w.L, S=w.S, dom=escg.circulant_dom(w.S, w.K), ex=w.ex,
                    sel=w.sel, rep=w.rep, seed=w.seed, replica=w.replica)
    tuned = autotune.apply(torch, p, "persistent")
    autotuned = tuned is not p
    p = tuned
    lat = torch.empty(w.L * w.L, dtype=torch.uint8, device="cuda")
    cnt = torch.empty((w.mcs + 1) * (w.S + 1), dtype=torch.int32,
                      device="cuda")
    escg.init(p, lat)
    escg.step_mcs(p, lat, 0, w.mcs, cnt)
    torch.cuda.synchronize()
    reps = max(1, min(5, args.steps))
    t0 = time.perf_counter()
    for _ in range(reps):
        escg.init(p, lat)
        escg.step_mcs(p, lat, 0, w.mcs, cnt)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    c = cnt.cpu().numpy().reshape(w.mcs + 1, w.S + 1)
    assert (c.sum(1) == w.L * w.L).all()
    return {"workload": "rps_L512_M1e-4_10000mcs (counts every MCS)",
            "site_updates_per_s": float(w.L) ** 2 * w.mcs / wall,
            "ms_per_run": wall * 1e3, "route": escg.last_route(),
            "tile_TH_TW_threads": escg.tile_plan(p, True),
            "tile_shape_autotuned": autotuned, "reps": reps}


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
    res = {"o1_one_thread": {"value": float(w.L) ** 2 * n1 / d1,
                              "unit": "site-updates/s",
                              "sample": f"L={w.L} RPSLS, {n1} MCS, "
                                        f"{d1:.1f} s"},
            "o2_all_cores": {"value": su / dall, "unit": "site-updates/s",
                             "cores": cores,
                             "sample": f"{cores} replicas of L={L} RPSLS "
                                       f"x {n} MCS, one per process, "
                                       f"{dall:.1f} s"},
           "host": host_cpu()}
    return res


def _o2_job(args):
    import oracle as O
    L, S, K, ex, seed, replica, n = args
    job = O.Job(L, S, O.circulant_matrix(S, K), ex, seed=seed,
                replica=replica)
    g = job.init()
    O.o2_run(job, g, 0, n, want_counts=False)
    return L * L * n


def cpu_jobs(workloads, batch_su_per_job):
    """Jobs/s of the oracle on every host core for the batched-replica and
    serving workloads: site-updates/s measured on all cores over a sample
    of each workload's jobs (every job truncated to a few MCS, one job per
    task), divided by the mean site-updates of one whole job (batch: from
    the GPU run's stopping times; serving: from the request table)."""
    import multiprocessing as mp
    cores = max(1, min(16, os.cpu_count() or 1))
    out = {"cores": cores, "kind": "oracle"}
    tab = workloads.batch_replicas()
    rng = np.random.default_rng(7)
    idx = rng.choice(len(tab), size=4 * cores, replace=False)
    tasks = [(int(tab.L[i]), 3, [1], float(tab.ex[i]), tab.seed, int(i), 40)
             for i in idx]
    t0 = time.perf_counter()
    with mp.Pool(cores) as pool:
        su = sum(pool.map(_o2_job, tasks))
    d = time.perf_counter() - t0
    out["batch"] = {"site_updates_per_s": su / d,
                    "jobs_per_s": su / d / batch_su_per_job
                    if batch_su_per_job else None,
                    "sample": f"{len(tasks)} random replicas x 40 MCS on "
                              f"{cores} processes, {d:.1f} s"}
    reqs = workloads.serving_requests()
    mean_su = float(np.mean([float(r.L) ** 2 * r.mcs for r in reqs]))
    pick = rng.choice(len(reqs), size=2 * cores, replace=False)
    tasks = [(reqs[i].L, reqs[i].S, list(reqs[i].K), reqs[i].ex, reqs[i].seed,
              0, 6) for i in pick]
    t0 = time.perf_counter()
    with mp.Pool(cores) as pool:
        su = sum(pool.map(_o2_job, tasks))
    d = time.perf_counter() - t0
    out["serving"] = {"site_updates_per_s": su / d,
                      "jobs_per_s": su / d / mean_su,
                      "sample": f"{len(tasks)} random requests x 6 MCS on "
                                f"{cores} processes, {d:.1f} s; mean job "
                                f"{mean_su:.3g} site-updates"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--skip-extras", action="store_true",
                    help="headline only (no batch, serving, cpu baseline)")
    ap.add_argument("--leg", choices=["batch", "serving"], default=None,
                    help="run only this leg (for profiling its kernels): "
                         "the batched replicas, or the server at "
                         "saturation (every request at t = 0)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="only run device-to-device copies of this many MiB "
                         "(reference for rocprofv3 byte counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU "
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
    if args.leg == "batch":
        print(json.dumps({"batch": batch(args, torch, escg, workloads)}),
              flush=True)
        return
    if args.leg == "serving":
        from paper_2508_16639_amd import serve
        r = serve.bench_serving(torch, escg, workloads, rates=(),
                                plain=False)
        print(json.dumps({"serving_capacity": r["capacity"]}), flush=True)
        return

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
                     "achieved_is": "algorithmic bytes (2 B per "
                                    "site-update) / kernel time, not "
                                    "measured HBM bandwidth",
                     "measured_hbm_GBs": (traffic / (h["kernel_ms"] * 1e-3)
                                          / 1e9 if traffic else None),
                     "binding_limit": "alu (integer VALU issue; the lattice "
                                      "stays in LDS, see the alu block)",
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
        log("[bench] rps L=512 (10000 MCS, counts every MCS)")
        out["rps_L512"] = rps512(args, torch, escg, workloads)
        log("[bench] serving")
        out["serving"] = serving(args, torch, escg, workloads)
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w)
        log("[bench] cpu context (O1, all-core O2)")
        out["cpu_context"] = cpu_context(w)
        out["cpu_context"]["jobs"] = cpu_jobs(
            workloads, out["batch"].get("su_per_job"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
