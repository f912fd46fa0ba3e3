"""Autotuner for the transform tile shapes.

Plan-wide knobs: pencils per x/y workgroup (8, 16, 32, 64), waves of rows per
z workgroup (1, 2, 4; 8 = one-wave workgroups with twice the lanes per row
in the z matvec), x slabs of the y-z-y chain (1, 2, 4, 8) and an occupancy
floor (1 or 4 waves per SIMD).  ``tune`` times one forward solve of a plan
for every plan-wide candidate and keeps the fastest; ``tune_passes`` then
gives each PCG pass its own (pencils, occupancy) by coordinate descent on
the whole forward solve's time.  Results are cached per (GPU architecture,
grid size, precision, batch class) in a JSON file; plans created through
``api.Plan`` apply the cached choice when they bind.
"""
from __future__ import annotations

import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(PKG, "schedules.json")
PENCILS = (8, 16, 32, 64)
Z_WAVES = (1, 2, 4, 8)
SLABS = (1, 2, 4, 8)
OCCUPANCY = (1, 4)
# PCG passes with their own tile shape, with the field volumes each moves
# per problem (for the achieved-bandwidth report)
PASSES = {"x_inv_grad": 5, "y_inv_grad": 5, "z_matvec": 7, "y_fwd_div": 5, "x_fwd_div": 7}


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
    """((pencils, z_waves, slabs, waves_per_simd), {pass: (pencils, waves)}) or None."""
    ent = load().get(key(arch, n, precision, batch))
    if not ent:
        return None
    sch = (int(ent["pencils"]), int(ent["z_waves"]), int(ent.get("slabs", 1)),
           int(ent.get("waves_per_simd", 1)))
    passes = {k: (int(v[0]), int(v[1])) for k, v in ent.get("passes", {}).items()}
    return sch, passes


def gpu_arch(device) -> str:
    import torch
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def _time_forward(plan, args, reps):
    import torch
    st = torch.cuda.current_stream(plan.device)
    plan.forward(*args)  # warm-up (also fixes the PCG chunking)
    torch.cuda.synchronize(plan.device)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        plan.forward(*args)
    e1.record(st)
    torch.cuda.synchronize(plan.device)
    return e0.elapsed_time(e1) / reps


def tune(plan, p, rho_f, k_f, m, reps: int = 2, candidates=None, verbose: bool = False):
    """Time plan.forward for every plan-wide (pencils, z_waves, slabs,
    waves_per_simd) candidate; set and return the fastest with the table of
    timings (ms)."""
    cands = candidates or [(c, w, s, o) for c in PENCILS for w in Z_WAVES for s in SLABS
                           for o in OCCUPANCY]
    times = {}
    for cand in cands:
        try:
            plan.set_schedule(*cand)
        except Exception:
            continue
        times[cand] = _median_forward(plan, (p, rho_f, k_f, m), reps)
        if verbose:
            print(f"  schedule {cand}: {times[cand]:.2f} ms", flush=True)
    best = min(times, key=times.get)
    plan.set_schedule(*best)
    return best, times


def _median_forward(plan, args, reps):
    ts = sorted(_time_forward(plan, args, reps) for _ in range(3))
    return ts[1]


def tune_passes(plan, p, rho_f, k_f, m, reps: int = 2, verbose: bool = False):
    """Per-pass (pencils, waves_per_simd) on top of the plan's current
    schedule, by coordinate descent on the whole forward solve (a pass's
    tile shape also changes its neighbours' cache behaviour, so passes are
    not timed alone).  A change is kept only if it saves more than 0.5%.
    Returns (passes, forward ms before, forward ms after)."""
    args = (p, rho_f, k_f, m)
    base = best_t = _median_forward(plan, args, reps)
    zw = plan.get_schedule()[1]
    chosen = {}
    # the wide z matvec (z_waves 8) has no per-pass variant
    names = [k for k in PASSES if not (k == "z_matvec" and zw == 8)]
    for name in names:
        if name == "z_matvec":
            # row layout in registers: single complex values or pairs
            opts = [(a, o) for a in (8, 16) for o in OCCUPANCY]
        else:
            opts = [(c, o) for c in PENCILS for o in OCCUPANCY]
        cur = best = plan.get_pass(name)
        for opt in opts:
            if opt == cur:
                continue
            try:
                plan.set_pass(name, *opt)
            except Exception:
                continue
            t = _median_forward(plan, args, reps)
            if verbose:
                print(f"  pass {name} {opt}: {t:.2f} ms", flush=True)
            if t < best_t * 0.995:
                best, best_t = opt, t
        plan.set_pass(name, *best)
        if best != cur:
            chosen[name] = best
        if verbose:
            print(f"  pass {name} -> {best} ({best_t:.2f} ms)", flush=True)
    return ({k: plan.get_pass(k) for k in names} if chosen else {}), base, best_t


def store(entries: dict, path: str | None = None) -> None:
    path = path or cache_path()
    tab = load(path)
    tab.update(entries)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(tab, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
