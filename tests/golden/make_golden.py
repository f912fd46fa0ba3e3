"""Write oracle reference values for the GPU parity tests at the
benchmark configurations (calls only the FP64 oracle and the input
generators).

    python tests/golden/make_golden.py config2      # 128^3 gradient
    python tests/golden/make_golden.py config3fwd   # 256^3 forward, sampled
    python tests/golden/make_golden.py config3grad  # 256^3 gradient + 2 GN products
    python tests/golden/make_golden.py config5hvp   # the 2 GN products alone

Outputs are small .npz files next to this script: scalars, the full
gradient vector and c(T) at a seeded sample of grid points.  The 256^3
runs switch the oracle's transforms to scipy.fft on several threads
(TG_ORACLE_FFT_WORKERS, default 6); they take a few hours.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import tumor  # noqa: E402
from paper_1907_07774_amd import inputs  # noqa: E402

NSAMPLE = 4096


def sample_idx(n, seed=123):
    rng = np.random.default_rng(seed)
    return rng.choice(n ** 3, NSAMPLE, replace=False)


def config2(rtol=1e-13):
    """128^3, 64 Gaussians, rho_f = 10, k_f = 0.1, T = 1, nt = 16; synthetic
    observation: threshold of a perturbed-p run."""
    n, nt, seed = 128, 16, 2
    pr = inputs.problem(n, 4, seed, nt=nt, rho_f=10.0, k_f=0.1)
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, nt, rtol=rtol)
    t0 = time.time()
    d = inputs.threshold_mask(tumor.forward(su, inputs.perturbed_p(pr.p, seed)).c[-1])
    J, g, tr = tumor.gradient(su, pr.p, d)
    idx = sample_idx(n)
    np.savez_compressed(os.path.join(HERE, "config2_128.npz"), n=n, nt=nt, seed=seed,
                        rho_f=pr.rho_f, k_f=pr.k_f, rtol=rtol, J=J, g_p=g.g_p, g_rho=g.g_rho,
                        g_k=g.g_k, idx=idx, cT=tr.c[-1].ravel()[idx],
                        cT_norm=np.linalg.norm(tr.c[-1]), d_idx=np.flatnonzero(d.ravel()),
                        its_fwd=np.array(tr.its), its_adj=np.array(g.its))
    print(f"config2 done in {time.time() - t0:.0f} s: J={J:.6e}", flush=True)


def config3fwd(rtol=1e-10):
    """256^3 forward of the benchmark problem (seed 0, 64 Gaussians, rho_f and
    k_f drawn from the seed, nt = 32): c(T) at sampled points."""
    n, nt, seed = 256, 32, 0
    pr = inputs.problem(n, 4, seed, nt=nt)
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, nt, rtol=rtol)
    t0 = time.time()
    c = tumor.phi(pr.p, pr.centres, pr.sigma, n)
    tau = 0.5 * su.dt
    its = []
    for _ in range(nt):  # the oracle's forward step, keeping only the state
        a = tumor.reaction(c, su.m, su.rho_f, tau)
        rhs = a + tau * su.k_f * tumor._A_m(su, a)
        b, it = tumor._cn_solve(su, rhs, a)
        c = tumor.reaction(b, su.m, su.rho_f, tau)
        its.append(it)
        print(f"  step {len(its)}/{nt}: {it} its, {time.time() - t0:.0f} s", flush=True)
    idx = sample_idx(n)
    np.savez_compressed(os.path.join(HERE, "config3_256_forward.npz"), n=n, nt=nt, seed=seed,
                        rho_f=pr.rho_f, k_f=pr.k_f, rtol=rtol, idx=idx, cT=c.ravel()[idx],
                        cT_norm=np.linalg.norm(c), cT_sum=c.sum(), its=np.array(its))
    print(f"config3fwd done in {time.time() - t0:.0f} s", flush=True)


def _log(t0, msg):
    print(f"[{time.time() - t0:7.0f} s] {msg}", flush=True)


def config3grad(rtol=1e-10):
    """256^3 gradient of the benchmark problem (seed 0, 64 Gaussians, rho_f
    and k_f drawn from the seed, T = 1, nt = 32), then the Gauss-Newton
    products of the first two of the eight benchmark directions about the
    same trajectory.  The observation is the oracle's own threshold of the
    perturbed-p run, stored bit-packed so the GPU tests and the benchmark
    evaluate exactly this misfit.  Two files: config3_256_grad.npz (written
    first) and config5_256_hvp.npz."""
    from oracle import spectral
    spectral.set_fft_workers(int(os.environ.get("TG_ORACLE_FFT_WORKERS", "6")))
    n, nt, seed = 256, 32, 0
    pr = inputs.problem(n, 4, seed, nt=nt)
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, nt, rtol=rtol)
    t0 = time.time()
    _log(t0, f"config3grad: rho_f={pr.rho_f:.6f} k_f={pr.k_f:.6f} rtol={rtol}")
    tr_obs = tumor.forward(su, inputs.perturbed_p(pr.p, seed))
    d = inputs.threshold_mask(tr_obs.c[-1])
    its_obs = list(tr_obs.its)
    del tr_obs
    _log(t0, f"observation: {int(d.sum())} voxels, {sum(its_obs)} its")
    tr = tumor.forward(su, pr.p)
    _log(t0, f"forward: {sum(tr.its)} its")
    J, lamT = tumor.misfit(su, tr.c[-1], d)
    g = tumor.vjp(su, tr, lamT)
    _log(t0, f"adjoint: {sum(g.its)} its, J={J:.10e}")
    idx = sample_idx(n)
    np.savez_compressed(os.path.join(HERE, "config3_256_grad.npz"), n=n, nt=nt, seed=seed,
                        rho_f=pr.rho_f, k_f=pr.k_f, rtol=rtol, J=J, g_p=g.g_p,
                        g_rho=g.g_rho, g_k=g.g_k, idx=idx, cT=tr.c[-1].ravel()[idx],
                        cT_norm=np.linalg.norm(tr.c[-1]), d_bits=np.packbits(d.ravel() > 0),
                        its_obs=np.array(its_obs), its_fwd=np.array(tr.its),
                        its_adj=np.array(g.its))
    del g, lamT
    V = inputs.hvp_directions(8, pr.p.size, 0)[:2]
    HV = []
    for i, v in enumerate(V):
        HV.append(tumor.gn_hvp(su, tr, v))
        _log(t0, f"GN product {i}: |Hv| = {np.linalg.norm(HV[-1]):.6e}")
    np.savez_compressed(os.path.join(HERE, "config5_256_hvp.npz"), n=n, nt=nt, seed=seed,
                        rho_f=pr.rho_f, k_f=pr.k_f, rtol=rtol, dir_seed=0, V=V,
                        HV=np.array(HV))
    _log(t0, "config3grad done")


def config5hvp(rtol=1e-10, dirs=(0, 1), name="config5_256_hvp.npz"):
    """The Gauss-Newton products of config3grad alone (its own forward
    trajectory of the benchmark problem) along benchmark directions `dirs`
    (indices into the eight of inputs.hvp_directions, seed 0): `name`."""
    from oracle import spectral
    spectral.set_fft_workers(int(os.environ.get("TG_ORACLE_FFT_WORKERS", "6")))
    n, nt, seed = 256, 32, 0
    pr = inputs.problem(n, 4, seed, nt=nt)
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, nt, rtol=rtol)
    t0 = time.time()
    tr = tumor.forward(su, pr.p)
    _log(t0, f"forward: {sum(tr.its)} its")
    V = inputs.hvp_directions(8, pr.p.size, 0)[list(dirs)]
    HV = []
    for i, v in zip(dirs, V):
        HV.append(tumor.gn_hvp(su, tr, v))
        _log(t0, f"GN product {i}: |Hv| = {np.linalg.norm(HV[-1]):.6e}")
    np.savez_compressed(os.path.join(HERE, name), n=n, nt=nt, seed=seed,
                        rho_f=pr.rho_f, k_f=pr.k_f, rtol=rtol, dir_seed=0,
                        dirs=np.array(dirs), V=V, HV=np.array(HV))
    _log(t0, "config5hvp done")


def config5hvp_d1(rtol=1e-10):
    """Direction 1 alone (for a second process next to config5hvp):
    config5_256_hvp_d1.npz."""
    config5hvp(rtol, dirs=(1,), name="config5_256_hvp_d1.npz")


if __name__ == "__main__":
    which = sys.argv[1:] or ["config2"]
    for w in which:
        globals()[w]()
