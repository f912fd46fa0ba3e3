"""Tune transform tile shapes on this GPU and store them in the schedule
cache (``autotune.cache_path()``, or --out).

    python -m paper_1907_07774_amd.tune_schedules --n 256 --precision fp32
"""
from __future__ import annotations

import argparse
import sys

import numpy as np
import torch

from . import api, autotune, inputs


def tune_case(n, precision, batch, nt, seed, verbose=True, candidates=None, per_pass=True):
    probs = [inputs.problem(n, 2 if n <= 64 else 4, seed + b, nt=nt) for b in range(batch)]
    cen = np.stack([q.centres for q in probs])
    plan = api.Plan(n, nt, cen, probs[0].sigma, rtol=1e-8, precision=precision, batch=batch,
                    schedule=(0, 0, 0, 0))
    dt = plan.dtype
    dev = plan.device
    m = torch.tensor(np.stack([q.m for q in probs]), dtype=dt, device=dev)
    p = torch.tensor(np.stack([q.p for q in probs]), dtype=torch.float64, device=dev)
    rho = torch.tensor([q.rho_f for q in probs], dtype=torch.float64, device=dev)
    kf = torch.tensor([q.k_f for q in probs], dtype=torch.float64, device=dev)
    if verbose:
        print(f"tuning n={n} {precision} batch={batch} nt={nt}", flush=True)
    best, times = autotune.tune(plan, p, rho, kf, m, verbose=verbose, candidates=candidates)
    passes, before, after = ({}, times[best], times[best])
    if per_pass:
        passes, before, after = autotune.tune_passes(plan, p, rho, kf, m, verbose=verbose)
        if verbose:
            print(f"  per-pass shapes: {before:.2f} -> {after:.2f} ms "
                  f"({'kept' if passes else 'dropped'})", flush=True)
    arch = autotune.gpu_arch(dev)
    k = autotune.key(arch, n, precision, batch)
    ent = {"pencils": best[0], "z_waves": best[1], "slabs": best[2],
           "waves_per_simd": best[3] if len(best) > 3 else 1,
           "ms": min(after, times[best]) if passes else times[best],
           "passes": {name: list(v) for name, v in passes.items()},
           "table_ms": {"x".join(map(str, k)): round(t, 4) for k, t in times.items()}}
    del plan
    torch.cuda.empty_cache()
    return k, ent


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[256])
    ap.add_argument("--precision", nargs="+", default=["fp32"])
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--nt", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--no-passes", action="store_true",
                    help="skip the per-pass refinement")
    ap.add_argument("--candidates", default=None,
                    help="comma-separated pencils x z_waves x slabs x waves_per_simd, "
                         "e.g. 16x1x1x1,32x1x1x4")
    a = ap.parse_args(argv)
    cands = None
    if a.candidates:
        cands = [tuple(int(v) for v in c.split("x")) for c in a.candidates.split(",")]
    entries = {}
    for n in a.n:
        for prec in a.precision:
            k, ent = tune_case(n, prec, a.batch, a.nt, a.seed, candidates=cands,
                               per_pass=not a.no_passes)
            entries[k] = ent
            print(f"{k}: pencils={ent['pencils']} z_waves={ent['z_waves']} slabs={ent['slabs']} "
                  f"waves_per_simd={ent['waves_per_simd']} passes={ent['passes']} "
                  f"({ent['ms']:.2f} ms)", flush=True)
    autotune.store(entries, a.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
