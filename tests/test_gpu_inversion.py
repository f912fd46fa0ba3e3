"""The inversion driver on the GPU gradient.

The GPU misfit equals the FP64 oracle's at the same (p, k_f); the driver's
weighted-l2 phase on it reaches the minimizer scipy's L-BFGS-B finds on the
oracle; the two-phase driver on the FP32-mixed path recovers a sparse
initial condition and k_f at 64^3.
"""
import numpy as np
import pytest
import torch
from scipy.optimize import minimize

from oracle import tumor
from paper_1907_07774_amd import api, inputs, inversion

from test_inversion_host import OracleMisfit, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case16():
    pr, p_true, d = oracle_problem()
    plan = api.Plan(pr.n, pr.nt, pr.centres, pr.sigma, rtol=1e-13, precision="fp64")
    return pr, p_true, d, inversion.GpuMisfit(plan, pr.m, d, pr.rho_f), OracleMisfit(pr, d)


def test_gpu_misfit_equals_oracle(case16):
    print("case inversion misfit 16^3", flush=True)
    pr, p_true, d, gpu, ora = case16
    rng = np.random.default_rng(4)
    for k in (0.0, 0.05, 0.2):
        p = rng.uniform(0, 1, pr.p.size)
        Dg, gpg, gkg = gpu(p, k)
        Do, gpo, gko = ora(p, k)
        assert abs(Dg - Do) < 1e-10 * abs(Do)
        assert np.linalg.norm(gpg - gpo) < 1e-9 * np.linalg.norm(gpo)
        assert abs(gkg - gko) < 1e-9 * max(abs(gko), 1e-300) + 1e-14


def test_l2_phase_on_gpu_matches_oracle_minimizer(case16):
    print("case inversion l2 16^3", flush=True)
    pr, p_true, d, gpu, ora = case16
    n = pr.p.size
    cfg = inversion.InversionConfig(beta_p=1e-4, opttol=1e-10, maxit_l2=300, skip_l1=True)
    p0 = np.full(n, 0.5)
    _, g_ref, _ = gpu(np.zeros(n), 0.05)
    r, p, k = inversion.l2_phase(gpu, p0, 0.05, np.ones(n), float(np.linalg.norm(g_ref)), cfg)
    assert r.converged

    def f(x):
        D, gp, gk = ora(x[:n], x[n])
        return D + 0.5e-4 * float(x[:n] @ x[:n]), np.concatenate([gp + 1e-4 * x[:n], [gk]])

    ref = minimize(f, np.concatenate([p0, [0.05]]), jac=True, method="L-BFGS-B",
                   bounds=[(None, None)] * n + [(1e-4, None)],
                   options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 1000})
    assert np.abs(p - ref.x[:n]).max() < 1e-5
    assert abs(k - ref.x[n]) < 1e-6


def test_two_phase_inversion_fp32_64():
    """Two adjacent active Gaussians (2 of 27; the paper's synthetic
    targets enable two nearby ones), rho_f = 10, k_f = 0.1, 64^3, nt = 8,
    FP32-mixed path, two l1 + l2 passes (the second l1 phase at the first
    l2 estimate of k_f): the misfit falls by three orders of magnitude, the
    active Gaussians are the largest coefficients, k_f comes back within
    10% and the last l2 phase meets its gradient tolerance."""
    print("case inversion two-phase fp32 64^3", flush=True)
    pr = inputs.problem(64, 3, 21, nt=8, rho_f=10.0, k_f=0.1)
    p_true = np.zeros_like(pr.p)
    p_true[[4, 13]] = (0.9, 0.7)
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, pr.nt, rtol=1e-12)
    d = tumor.forward(su, p_true).c[-1]
    plan = api.Plan(64, pr.nt, pr.centres, pr.sigma, rtol=1e-8, precision="fp32")
    obj = inversion.GpuMisfit(plan, pr.m, d, pr.rho_f)
    cfg = inversion.InversionConfig(bisections=4, maxit_gist=40, opttol=1e-4, maxit_l2=150,
                                    outer=2)
    res = inversion.invert(obj, pr.p.size, cfg)
    D0 = obj(np.zeros(pr.p.size), 0.05)[0]
    print(f"misfit {res.misfit:.3e} (D0 {D0:.3e}) k_f {res.k_f:.4f} "
          f"top {np.argsort(-np.abs(res.p))[:3]} evals {res.evaluations}", flush=True)
    assert obj.failures == 0
    assert res.converged
    assert res.misfit < 1e-3 * D0
    assert set(np.argsort(-np.abs(res.p))[:2]) == {4, 13}
    assert abs(res.k_f - 0.1) < 0.01
    del plan
    torch.cuda.empty_cache()
