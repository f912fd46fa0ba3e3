"""Degenerate and boundary cases of the forward/adjoint path on the GPU
against the FP64 oracle, through the C-ABI: the smallest grid, a single
time step with a checkpoint stride beyond it, a single Gaussian, a zero
initial condition (c = 0 for all t) and a field without white matter
(m = 0: no diffusion and no reaction, so c(T) = Phi p and the k_f and
rho_f gradients vanish)."""
import numpy as np
import pytest

from oracle import tumor
from paper_1907_07774_amd import api, inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def scaled(pr):
    mx = tumor.phi(pr.p, pr.centres, pr.sigma, pr.n).max()
    return pr.p / max(mx, 1.0)


def both(pr, p, d, precision="fp64", ckpt=0, rtol=1e-13):
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, pr.nt, rtol=1e-13)
    J, g, tr = tumor.gradient(su, p, d)
    plan = api.Plan(pr.n, pr.nt, pr.centres, pr.sigma, rtol=rtol, precision=precision,
                    ckpt_stride=ckpt)
    cT = plan.forward(p, pr.rho_f, pr.k_f, pr.m).cpu().numpy()
    Jg, gp, gr, gk = plan.adjoint_misfit(d)
    assert plan.stats().status_bits == 0
    return (J, g, tr), (cT, float(Jg), gp.cpu().numpy(), float(gr), float(gk))


def check(ref, got, tol):
    (J, g, tr), (cT, Jg, gp, gr, gk) = ref, got
    assert rel(cT, tr.c[-1]) < tol
    assert abs(Jg - J) < tol * abs(J)
    assert rel(gp, g.g_p) < tol
    assert abs(gr - g.g_rho) < tol * abs(g.g_rho)
    assert abs(gk - g.g_k) < tol * abs(g.g_k)


@pytest.mark.parametrize("ckpt", [0, 2])
def test_smallest_grid_gradient_fp64(ckpt):
    print(f"case edge n=8 ckpt={ckpt}", flush=True)
    pr = inputs.problem(8, 2, 31, nt=3, rho_f=4.0, k_f=0.1, sigma=0.6)
    p = scaled(pr)
    d = inputs.random_field(8, 31)
    check(*both(pr, p, d, ckpt=ckpt), 1e-10)


@pytest.mark.parametrize("precision,tol,ckpt", [("fp64", 1e-10, 4), ("fp32", 1e-4, 3)])
def test_single_step_with_stride_beyond_it(precision, tol, ckpt):
    """nt = 1 with a checkpoint stride larger than nt: no segment to
    recompute, the adjoint runs from the one stored state."""
    print(f"case edge nt=1 {precision}", flush=True)
    pr = inputs.problem(32, 2, 32, nt=1, rho_f=6.0, k_f=0.2)
    p = scaled(pr)
    d = inputs.threshold_mask(tumor.forward(
        tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, 1, rtol=1e-10),
        inputs.perturbed_p(p, 32)).c[-1])
    check(*both(pr, p, d, precision, ckpt, 1e-13 if precision == "fp64" else 1e-8), tol)


def test_single_gaussian_fp64():
    print("case edge n_p=1", flush=True)
    pr = inputs.problem(32, 1, 33, nt=4, rho_f=8.0, k_f=0.1)
    assert pr.p.size == 1
    p = scaled(pr)
    d = inputs.random_field(32, 33)
    check(*both(pr, p, d, ckpt=3), 1e-10)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_zero_initial_condition(precision):
    """p = 0: every solve has a zero right-hand side and stops before its
    first iteration; c(T) = 0, the rho_f and k_f gradients are 0 and the p
    gradient is Phi^T of the adjoint of -h^3 d."""
    print(f"case edge p=0 {precision}", flush=True)
    pr = inputs.problem(32, 2, 34, nt=4, rho_f=8.0, k_f=0.1)
    p = np.zeros_like(pr.p)
    d = inputs.random_field(32, 34)
    (J, g, tr), (cT, Jg, gp, gr, gk) = both(pr, p, d, precision, 2,
                                            1e-13 if precision == "fp64" else 1e-8)
    assert np.all(cT == 0.0) and np.all(tr.c[-1] == 0.0)
    assert g.g_rho == 0.0 and g.g_k == 0.0 and gr == 0.0 and gk == 0.0
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert abs(Jg - J) < tol * J
    assert rel(gp, g.g_p) < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_no_white_matter(precision):
    """m = 0: c(T) = Phi p (the reaction factor is 1 and the diffusion
    operator 0) and only the p gradient is nonzero."""
    print(f"case edge m=0 {precision}", flush=True)
    pr = inputs.problem(32, 2, 35, nt=4, rho_f=8.0, k_f=0.1)
    pr.m[...] = 0.0
    p = scaled(pr)
    d = inputs.random_field(32, 35)
    (J, g, tr), (cT, Jg, gp, gr, gk) = both(pr, p, d, precision, 0,
                                            1e-13 if precision == "fp64" else 1e-8)
    c0 = tumor.phi(p, pr.centres, pr.sigma, 32)
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert rel(tr.c[-1], c0) < 1e-14
    assert rel(cT, c0) < tol
    assert g.g_rho == 0.0 and g.g_k == 0.0 and gr == 0.0 and gk == 0.0
    assert abs(Jg - J) < tol * J
    assert rel(gp, g.g_p) < (1e-10 if precision == "fp64" else 1e-5)
