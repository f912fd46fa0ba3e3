"""Autotuner for the transform tile shapes.

The x/y passes take C pencils per workgroup (C in 8, 16, 32) and the z pass
takes 1, 2 or 4 waves of rows per workgroup.  ``tune`` times one forward
solve of a plan for every candidate pair and keeps the fastest; results are
cached per (GPU architecture, grid size, precision, batch) in a JSON file.
Plans created through ``api.Plan`` apply the cached choice when they bind.
"""
from __future__ import annotations

import json
import os
import time

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(PKG, "schedules.json")
PENCILS = (8, 16, 32)
Z_WAVES = (1, 2, 4, 8)
SLABS = (1, 2, 4, 8)
OCCUPANCY = (1, 4)


def cache_path() -> str:
    return os.environ.get("TUMORGRAD_SCHEDULES", DEFAULT_CACHE)


def key(arch: str, n: int, precision: str, batch: int) -> str:
    bclass = 1 if batch <= 1 else (8 if batch <= 8 else 64)
    return f"{arch}/n{n}/{precision}/b{bclass}"


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(arch: str, n: int, precision: str, batch: int):
    ent = load().get(key(arch, n, precision, batch))
    if not ent:
        return None
    return (int(ent["pencils"]), int(ent["z_waves"]), int(ent.get("slabs", 1)),
            int(ent.get("waves_per_simd", 1)))


def gpu_arch(device) -> str:
    import torch
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def tune(plan, p, rho_f, k_f, m, reps: int = 2, candidates=None, verbose: bool = False):
    """Time plan.forward for every (pencils, z_waves, slabs, waves_per_simd)
    candidate; set and return the fastest with the table of timings (ms)."""
    import torch
    cands = candidates or [(c, w, s, o) for c in PENCILS for w in Z_WAVES for s in SLABS
                           for o in OCCUPANCY]
    times = {}
    st = torch.cuda.current_stream(plan.device)
    for cand in cands:
        try:
            plan.set_schedule(*cand)
        except Exception:
            continue
        plan.forward(p, rho_f, k_f, m)  # warm-up (also fixes the PCG chunking)
        torch.cuda.synchronize(plan.device)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            plan.forward(p, rho_f, k_f, m)
        e1.record(st)
        torch.cuda.synchronize(plan.device)
        times[cand] = e0.elapsed_time(e1) / reps
        if verbose:
            print(f"  schedule {cand}: {times[cand]:.2f} ms", flush=True)
    best = min(times, key=times.get)
    plan.set_schedule(*best)
    return best, times


def store(entries: dict, path: str | None = None) -> None:
    path = path or cache_path()
    tab = load(path)
    tab.update(entries)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(tab, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
