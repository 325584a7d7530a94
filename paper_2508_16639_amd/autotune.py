"""Autotuner for the launch choices of the tiled and batched kernels.

Every choice it makes (tile shape, workgroup size, resident workgroups per
compute unit) selects among kernels that give the same bytes, so tuning
never changes results, only speed.  Results are cached in a JSON file keyed
by architecture, compute-unit count, kernel, lattice side (or side mix) and
species class (S <= 7 or S > 7: the two kernel instantiations), and applied
per call through the job's launch choices (escg.Params.with_launch).

Kernels tuned:
  persistent  the persistent tiled kernel of one large lattice: tile shape
              (TH, TW) and workgroup size cap (threads), which together set
              the tiles and waves per CU;
  step        the per-MCS tiled kernel (escg_step_batch with route "tiled"):
              tile shape and workgroup size cap;
  multi       the multi-job persistent kernel (escg_step_batch): the tile
              shape of one lattice side, timed with as many copies of the
              job as fill the GPU (its workgroups have a fixed 1024 threads,
              one per CU);
  batch       the LDS-resident batch kernel: workgroup size and resident
              workgroups per CU, for a mix of lattice sides.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                     "autotune_cache.json")


def candidates(L: int, cus: int, max_tiles_per_cu: int = 3,
               min_tiles: int = 0) -> List[Tuple[int, int]]:
    """Tile shapes (TH, TW) dividing L, TW % 8 == 0, TH even >= 4, with
    between min_tiles (default cus/8) and max_tiles_per_cu*cus tiles and at
    most 512 per side."""
    out = []
    if L % 8:
        return out
    for TW in range(8, min(L, 512) + 1, 8):
        if L % TW:
            continue
        for TH in range(4, min(L, 512) + 1, 2):
            if L % TH:
                continue
            T = (L // TH) * (L // TW)
            if (min_tiles or max(1, cus // 8)) <= T <= max_tiles_per_cu * cus:
                out.append((TH, TW))
    return out


def device_key(torch) -> str:
    """Architecture and compute-unit count: what the choices depend on
    (marketing names differ between driver versions)."""
    prop = torch.cuda.get_device_properties(0)
    arch = getattr(prop, "gcnArchName", "") or torch.cuda.get_device_name(0)
    return f"{arch.split(':')[0]}|cus={prop.multi_processor_count}"


def key(torch, kernel: str, L, S: int) -> str:
    """Cache key; L is a side or a tuple of sides (a batch's mix)."""
    side = ",".join(str(int(x)) for x in L) if isinstance(L, (tuple, list)) \
        else str(int(L))
    return f"{device_key(torch)}|{kernel}|L={side}|S<=7={int(S <= 7)}"


_memo = {"mtime": None, "data": {}}


def load_cache() -> Dict[str, dict]:
    """The cache file's records (re-read only when the file changes)."""
    if not os.path.exists(CACHE):
        return {}
    mt = os.path.getmtime(CACHE)
    if _memo["mtime"] != mt:
        with open(CACHE) as f:
            _memo["data"] = json.load(f)
        _memo["mtime"] = mt
    return _memo["data"]


def _save(k: str, rec: dict) -> None:
    cache = dict(load_cache())
    cache[k] = rec
    with open(CACHE, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def lookup(torch, kernel: str, L, S: int) -> Optional[dict]:
    return load_cache().get(key(torch, kernel, L, S))


def launch_choice(rec: Optional[dict]) -> dict:
    """escg.Params.with_launch keywords of a cache record ({} if none)."""
    if not rec:
        return {}
    out = {}
    if rec.get("TH"):
        out["tile"] = (rec["TH"], rec["TW"])
    if rec.get("threads"):
        out["threads"] = rec["threads"]
    if rec.get("wg_per_cu"):
        out["wg_per_cu"] = rec["wg_per_cu"]
    return out


def apply(torch, p, kernel: str = "persistent", L=None):
    """p with the cached choices of `kernel` for its side (or the side mix
    L), unchanged if none are cached."""
    kw = launch_choice(lookup(torch, kernel, p.L if L is None else L, p.S))
    return p.with_launch(**kw) if kw else p


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune_tiled(torch, escg, L: int, S: int, K=None, ex: float = 1.0,
               kernel: str = "persistent", n_mcs: int = 400, reps: int = 3,
               limit: int = 16, threads=(512, 768, 1024),
               save: bool = True) -> dict:
    """Times the planner's own choice and up to `limit` tile shapes (least
    halo overhead first) times the workgroup size caps `threads` on the
    persistent ("persistent") or per-MCS ("step") tiled kernel, n_mcs MCS
    per run (long enough that per-launch costs do not decide), and records
    the fastest."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    cands = candidates(L, cus)
    cands.sort(key=lambda s: ((s[0] + 8) * (s[1] + 16)) / (s[0] * s[1]))
    cands = cands[:limit]
    if kernel == "step":
        threads = tuple(t for t in threads if t <= 512) or (512,)
    if K is None:
        K = (1,) if S == 3 else tuple(range(1, (S + 1) // 2 + 1))
    route = "persistent" if kernel == "persistent" else "tiled"
    base = escg.Params(L=L, S=S, dom=escg.circulant_dom(S, K), ex=ex, seed=7,
                       route=route)
    lat = torch.empty(L * L, dtype=torch.uint8, device="cuda")
    cnt = torch.empty((n_mcs + 1) * (S + 1), dtype=torch.int32, device="cuda")
    escg.init(base, lat)
    results = []
    seen = set()
    trials = [(None, 0)] + [(c, nt) for c in cands for nt in threads]
    for shape, nt in trials:
        p = base.with_launch(tile=shape, threads=nt)
        plan = escg.tile_plan(p, kernel == "persistent")
        if plan is None or plan in seen:
            continue  # does not fit, or the same plan as another cap
        seen.add(plan)
        try:
            dt = _time(lambda: escg.step_mcs(p, lat, 0, n_mcs, cnt), reps)
        except escg.EscgError:
            continue
        results.append({"TH": plan[0], "TW": plan[1], "threads": plan[2],
                        "us_per_mcs": dt / n_mcs * 1e6,
                        "planner": shape is None})
    escg.async_status()
    if not results:
        return {}
    win = min(results, key=lambda r: r["us_per_mcs"])
    rec = dict(win, n_mcs=n_mcs,
               tried=sorted(results, key=lambda r: r["us_per_mcs"])[:8])
    if save:
        _save(key(torch, kernel, L, S), rec)
    return rec


def tune_multi(torch, escg, L: int, S: int, K=None, ex: float = 1.0,
               n_mcs: int = 200, reps: int = 3, limit: int = 12,
               save: bool = True) -> dict:
    """Times escg_step_batch's persistent launches on copies of one job of
    side L for up to `limit` tile shapes (least halo overhead first) whose
    region takes the balanced quad list at 1024 threads (at most three quads
    per thread and pass; larger regions fall back to the slower column walk
    and make launches long and coarse for a server), as many copies as one
    launch holds, and records the shape with the most site-updates per
    second."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count

    def list_fits(TH, TW):
        return ((TH + 8) // 2) * ((TW + 16) // 8) <= 3 * 1024

    cands = [c for c in candidates(L, cus, max_tiles_per_cu=1, min_tiles=1)
             if (L // c[0]) * (L // c[1]) <= cus and list_fits(*c)]
    cands.sort(key=lambda s: ((s[0] + 8) * (s[1] + 16)) / (s[0] * s[1]))
    cands = [None] + cands[:limit]  # None: the planner's own shape
    if K is None:
        K = (1,) if S == 3 else tuple(range(1, (S + 1) // 2 + 1))
    base = escg.Params(L=L, S=S, dom=escg.circulant_dom(S, K), ex=ex, seed=7)
    results = []
    seen = set()
    for shape in cands:
        plan = escg.tile_plan(base.with_launch(tile=shape), "multi")
        if plan is None or plan[:2] in seen:
            continue
        seen.add(plan[:2])
        TH, TW = plan[0], plan[1]
        T = (L // TH) * (L // TW)
        k = max(1, cus // T)
        ps = [base.with_launch(tile=shape) for _ in range(k)]
        ps = [dataclasses.replace(q, replica=i) for i, q in enumerate(ps)]
        lats = [torch.empty(L * L, dtype=torch.uint8, device="cuda")
                for _ in range(k)]
        for q, t in zip(ps, lats):
            escg.init(q, t)
        try:
            dt = _time(lambda: escg.step_batch(ps, lats, [0] * k,
                                               [n_mcs] * k), reps)
        except escg.EscgError:
            continue
        if escg.last_route() != "persistent":
            continue
        results.append({"TH": TH, "TW": TW, "copies": k,
                        "su_per_s": k * float(L) ** 2 * n_mcs / dt,
                        "planner": shape is None})
    escg.async_status()
    if not results:
        return {}
    win = max(results, key=lambda r: r["su_per_s"])
    rec = dict(win, n_mcs=n_mcs,
               tried=sorted(results, key=lambda r: -r["su_per_s"])[:8])
    if save:
        _save(key(torch, "multi", L, S), rec)
    return rec


def tune_batch(torch, escg, params: Sequence, offsets, max_mcs, mode: int,
               sides, reps: int = 2, threads=(128, 256, 384, 512),
               wg_per_cu=(0, 1, 2, 3, 4), save: bool = True) -> dict:
    """Times escg.batch_run on the given batch (its own parameters, offsets
    and budgets) for each workgroup size and resident workgroups per CU, and
    records the fastest under the side mix `sides`."""
    n = len(params)
    end = max(int(o) + int(p.L) ** 2 for o, p in zip(offsets, params))
    buf = torch.empty(end, dtype=torch.uint8, device="cuda")
    res = torch.empty(n * escg.BATCH_RESULT_WORDS, dtype=torch.int32,
                      device="cuda")
    results = []
    for nt in threads:
        for w in wg_per_cu:
            ps = [params[0].with_launch(threads=nt, wg_per_cu=w)] + \
                list(params[1:])
            dt = _time(lambda: escg.batch_run(ps, offsets, buf, max_mcs, mode,
                                              True, res), reps)
            results.append({"threads": nt, "wg_per_cu": w,
                            "jobs_per_s": n / dt})
    win = max(results, key=lambda r: r["jobs_per_s"])
    rec = dict(win, n_jobs=n,
               tried=sorted(results, key=lambda r: -r["jobs_per_s"])[:8])
    if save:
        _save(key(torch, "batch", tuple(sides), params[0].S), rec)
    return rec


def tune_replica_batch(torch, escg, workloads, save: bool = True) -> dict:
    """tune_batch on the batched-replica workload (4096 RPS replicas, L in
    {64, 128, 192, 256}, first extinction or 20 L MCS)."""
    tab = workloads.batch_replicas()
    dom = escg.circulant_dom(3, [1])
    params, offs, off = [], [], 0
    for r in range(len(tab)):
        L = int(tab.L[r])
        params.append(escg.Params(L=L, S=3, dom=dom, ex=float(tab.ex[r]),
                                  seed=tab.seed, replica=r))
        offs.append(off)
        off += L * L
    sides = tuple(sorted(set(int(x) for x in tab.L)))
    return tune_batch(torch, escg, params, offs, tab.max_mcs,
                      escg.STOP_FIRST_EXTINCTION, sides, reps=1, save=save)


if __name__ == "__main__":
    # kernel:L:S arguments ("persistent:3200:5", "step:1600:3",
    # "multi:1600:5"), or "batch" for the batched-replica workload
    import sys
    import torch
    from paper_2508_16639_amd import escg, workloads
    for arg in sys.argv[1:] or ["persistent:3200:5"]:
        if arg == "batch":
            rec = tune_replica_batch(torch, escg, workloads)
        else:
            kern, L, S = arg.split(":")
            if kern == "multi":
                rec = tune_multi(torch, escg, int(L), int(S))
            else:
                rec = tune_tiled(torch, escg, int(L), int(S), kernel=kern)
        print(arg, json.dumps({k: v for k, v in rec.items() if k != "tried"}),
              flush=True)
