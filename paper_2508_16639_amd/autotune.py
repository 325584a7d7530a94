"""Tile-shape autotuner for the tiled kernels.

For a lattice side L and species count S it times the persistent kernel
(one cooperative launch, LDS-resident tiles) on candidate tile shapes and
keeps the fastest.  Results are cached in a JSON file keyed by device name,
L and whether S <= 7 (the two kernel instantiations), and applied with
escg.set_tile_shape.  Every shape gives the same bytes, so tuning never
changes results.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional, Tuple

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                     "autotune_cache.json")


def candidates(L: int, cus: int, max_tiles_per_cu: int = 3
               ) -> List[Tuple[int, int]]:
    """Tile shapes (TH, TW) dividing L, TW % 8 == 0, TH even >= 4, with
    between cus/2 and max_tiles_per_cu*cus tiles and at most 512 per side."""
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
            if cus // 2 <= T <= max_tiles_per_cu * cus:
                out.append((TH, TW))
    return out


def device_key(torch) -> str:
    """Architecture and compute-unit count: what the tile shape depends on
    (marketing names differ between driver versions)."""
    prop = torch.cuda.get_device_properties(0)
    arch = getattr(prop, "gcnArchName", "") or torch.cuda.get_device_name(0)
    return f"{arch.split(':')[0]}|cus={prop.multi_processor_count}"


def _key(torch, L: int, S: int) -> str:
    return f"{device_key(torch)}|L={L}|S<=7={int(S <= 7)}"


def load_cache() -> Dict[str, dict]:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def apply_cached(torch, escg, L: int, S: int) -> Optional[Tuple[int, int]]:
    rec = load_cache().get(_key(torch, L, S))
    if not rec:
        return None
    escg.set_tile_shape(L, rec["TH"], rec["TW"])
    return rec["TH"], rec["TW"]


def tune(torch, escg, L: int, S: int, K=None, ex: float = 1.0,
         n_mcs: int = 40, reps: int = 2, limit: int = 24,
         save: bool = True) -> dict:
    """Times up to `limit` candidate shapes (those with the least halo
    overhead first) and records the fastest."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    cands = candidates(L, cus)
    cands.sort(key=lambda s: ((s[0] + 8) * (s[1] + 16)) / (s[0] * s[1]))
    cands = cands[:limit]
    if K is None:
        K = (1,) if S == 3 else tuple(range(1, (S + 1) // 2 + 1))
    p = escg.Params(L=L, S=S, dom=escg.circulant_dom(S, K), ex=ex, seed=7)
    lat = torch.empty(L * L, dtype=torch.uint8, device="cuda")
    cnt = torch.empty((n_mcs + 1) * (S + 1), dtype=torch.int32, device="cuda")
    escg.init(p, lat)
    old_min = escg.persistent_min_L()
    escg.set_persistent_min_L(0)
    results = []
    try:
        for TH, TW in cands:
            escg.set_tile_shape(L, TH, TW)
            if escg.tile_plan(L, S, True) != None and \
                    escg.tile_plan(L, S, True)[:2] != (TH, TW):
                continue  # does not fit the device
            escg.step_mcs(p, lat, 0, 2, cnt)
            torch.cuda.synchronize()
            if escg.last_route() != "persistent":
                continue
            best = float("inf")
            for _ in range(reps):
                t0 = time.perf_counter()
                escg.step_mcs(p, lat, 0, n_mcs, cnt)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            results.append({"TH": TH, "TW": TW,
                            "us_per_mcs": best / n_mcs * 1e6})
    finally:
        escg.set_tile_shape(L, 0, 0)
        escg.set_persistent_min_L(old_min)
    escg.async_status()
    if not results:
        return {}
    win = min(results, key=lambda r: r["us_per_mcs"])
    rec = {"TH": win["TH"], "TW": win["TW"],
           "us_per_mcs": win["us_per_mcs"], "n_mcs": n_mcs,
           "tried": sorted(results, key=lambda r: r["us_per_mcs"])[:8]}
    if save:
        cache = load_cache()
        cache[_key(torch, L, S)] = rec
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return rec


if __name__ == "__main__":
    import sys
    import torch
    from paper_2508_16639_amd import escg
    for arg in sys.argv[1:] or ["3200:5"]:
        L, S = (int(x) for x in arg.split(":"))
        print(L, S, json.dumps(tune(torch, escg, L, S)), flush=True)
