"""The inversion driver's optimizers, pinned on the CPU.

- Moré–Thuente line search: the strong Wolfe conditions and the evaluation
  counts their paper reports for its six test functions (Moré and Thuente,
  ACM TOMS 20, 1994, Tables 1-6), which a wrong interpolation or update
  rule changes.
- L-BFGS: the minimizer of Rosenbrock's function and of the tumor misfit
  (the FP64 oracle at 16^3) against scipy's L-BFGS-B.
- GIST: the l1-penalized least-squares minimizer against scikit-learn's
  coordinate-descent Lasso, and the l1-penalized tumor misfit against
  L-BFGS-B on the split p = u - v, u, v >= 0.
- Hoyer measure closed forms; the full two-phase driver on the oracle.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize, rosen, rosen_der

from oracle import tumor
from paper_1907_07774_amd import inputs, inversion, optim


def _f1(beta=2.0):
    return lambda a: (-a / (a * a + beta), (a * a - beta) / (a * a + beta) ** 2)


def _f2(beta=0.004):
    return lambda a: ((a + beta) ** 5 - 2 * (a + beta) ** 4,
                      5 * (a + beta) ** 4 - 8 * (a + beta) ** 3)


def _f3(beta=0.01, l=39):
    def phi(a):
        if a <= 1 - beta:
            v, d = 1 - a, -1.0
        elif a >= 1 + beta:
            v, d = a - 1, 1.0
        else:
            v, d = (a - 1) ** 2 / (2 * beta) + beta / 2, (a - 1) / beta
        return (v + 2 * (1 - beta) / (l * math.pi) * math.sin(l * math.pi * a / 2),
                d + (1 - beta) * math.cos(l * math.pi * a / 2))
    return phi


def _yanai(b1, b2):
    g = lambda b: math.sqrt(1 + b * b) - b

    def phi(a):
        r1, r2 = math.sqrt((1 - a) ** 2 + b2 * b2), math.sqrt(a * a + b1 * b1)
        return g(b1) * r1 + g(b2) * r2, g(b1) * (a - 1) / r1 + g(b2) * a / r2
    return phi


# (function, ftol, gtol, evaluations for initial steps 1e-3, 1e-1, 1e1, 1e3)
MT_CASES = [
    (_f1(), 1e-3, 0.1, (6, 3, 1, 4)),
    (_f2(), 0.1, 0.1, (12, 8, 8, 11)),
    (_f3(), 0.1, 0.1, (12, 12, 10, 13)),
    (_yanai(0.001, 0.001), 0.001, 0.001, (4, 1, 3, 4)),
    (_yanai(0.01, 0.001), 0.001, 0.001, (6, 3, 7, 8)),
    (_yanai(0.001, 0.01), 0.001, 0.001, (13, 11, 8, 11)),
]


@pytest.mark.parametrize("case", range(len(MT_CASES)))
def test_more_thuente_matches_published_counts(case):
    phi, ftol, gtol, counts = MT_CASES[case]
    f0, g0 = phi(0.0)
    for a0, want in zip((1e-3, 1e-1, 1e1, 1e3), counts):
        stp, f, g, nfev, info = optim.more_thuente(phi, f0, g0, stp=a0, ftol=ftol, gtol=gtol)
        assert info == "ok"
        assert f <= f0 + ftol * stp * g0 and abs(g) <= gtol * abs(g0)
        assert nfev == want, (case, a0, nfev)


def test_more_thuente_rejects_ascent():
    with pytest.raises(ValueError):
        optim.more_thuente(lambda a: (a, 1.0), 0.0, 1.0)


def test_lbfgs_rosenbrock():
    r = optim.lbfgs(lambda x: (rosen(x), rosen_der(x)), np.full(10, -1.2), gtol_rel=1e-10,
                    maxit=500)
    assert r.converged
    assert np.abs(r.x - 1.0).max() < 1e-6


def test_gist_matches_sklearn_lasso():
    from sklearn.linear_model import Lasso
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 12))
    x_true = np.zeros(12)
    x_true[[1, 5, 9]] = (2.0, -1.5, 0.7)
    b = A @ x_true + 0.05 * rng.standard_normal(40)
    beta = 2.0
    fg = lambda x: (0.5 * float((A @ x - b) @ (A @ x - b)), A.T @ (A @ x - b))
    r = optim.gist(fg, np.zeros(12), beta, tau_j=1e-16, maxit=20000)
    ref = Lasso(alpha=beta / 40, fit_intercept=False, tol=1e-14, max_iter=1000000).fit(A, b)
    assert np.abs(r.x - ref.coef_).max() < 1e-6
    assert set(np.flatnonzero(r.x)) == set(np.flatnonzero(ref.coef_))


def test_soft_threshold_and_hoyer():
    v = np.array([-3.0, -0.5, 0.2, 2.0])
    assert np.array_equal(optim.soft_threshold(v, 1.0), [-2.0, 0.0, 0.0, 1.0])
    assert optim.hoyer(np.array([0, 0, 5.0, 0])) == 1.0
    assert abs(optim.hoyer(np.full(7, -2.0))) < 1e-15
    assert abs(optim.hoyer(np.array([1.0, 1.0, 0, 0])) - 2 / 3) < 1e-15


# ---------------------------------------------------- tumor misfit (oracle)
def oracle_problem(n=16, nt=4):
    """Synthetic data from a sparse initial condition (two of the eight
    Gaussians active, as in the paper's synthetic targets)."""
    pr = inputs.problem(n, 2, 11, nt=nt, rho_f=8.0, k_f=0.15)
    p_true = np.zeros_like(pr.p)
    p_true[[2, 5]] = (0.8, 0.6)
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, nt, rtol=1e-13)
    d = tumor.forward(su, p_true).c[-1]
    return pr, p_true, d


class OracleMisfit:
    """D(p, k_f) and its gradient from the FP64 oracle."""

    def __init__(self, pr, d):
        self.pr, self.d = pr, d

    def __call__(self, p, k_f):
        pr = self.pr
        su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, float(k_f), pr.nt, rtol=1e-13)
        J, g, _ = tumor.gradient(su, np.asarray(p), self.d)
        return float(J), np.asarray(g.g_p, dtype=np.float64), float(g.g_k)


@pytest.fixture(scope="module")
def oracle_case():
    pr, p_true, d = oracle_problem()
    return pr, p_true, d, OracleMisfit(pr, d)


def test_l2_phase_matches_lbfgsb_minimizer(oracle_case):
    """The driver's L-BFGS + Moré–Thuente reaches the same minimizer of
    D + beta_p/2 |p|^2 over (p, k_f) as scipy's L-BFGS-B."""
    pr, p_true, d, obj = oracle_case
    cfg = inversion.InversionConfig(beta_p=1e-4, opttol=1e-10, maxit_l2=300, skip_l1=True)
    n = pr.p.size
    w = np.ones(n)
    p0 = np.full(n, 0.5)
    _, g_ref, _ = obj(np.zeros(n), 0.05)
    r, p, k = inversion.l2_phase(obj, p0, 0.05, w, float(np.linalg.norm(g_ref)), cfg)
    assert r.converged

    def f(x):
        D, gp, gk = obj(x[:n], x[n])
        return D + 0.5e-4 * float(x[:n] @ x[:n]), np.concatenate([gp + 1e-4 * x[:n], [gk]])

    ref = minimize(f, np.concatenate([p0, [0.05]]), jac=True, method="L-BFGS-B",
                   bounds=[(None, None)] * n + [(1e-4, None)],
                   options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 1000})
    assert np.abs(p - ref.x[:n]).max() < 1e-5
    assert abs(k - ref.x[n]) < 1e-6
    # the data were generated from (p_true, k_f = 0.15): the minimizer is close
    assert abs(k - 0.15) < 0.01


def test_gist_fixed_beta_matches_split_lbfgsb(oracle_case):
    """GIST on D(p) + beta ||p||_1 (k_f fixed) against L-BFGS-B on the
    smooth split p = u - v, u, v >= 0, whose minimizer is the same."""
    pr, p_true, d, obj = oracle_case
    n = pr.p.size
    k = 0.15
    fg = lambda p: obj(p, k)[:2]
    _, g0 = fg(np.zeros(n))
    beta = 0.05 * float(np.abs(g0).max())
    r = optim.gist(fg, np.zeros(n), beta, tau_j=1e-14, maxit=3000)

    def f(x):
        u, v = x[:n], x[n:]
        D, g = fg(u - v)
        return D + beta * float(u.sum() + v.sum()), np.concatenate([g + beta, -g + beta])

    ref = minimize(f, np.zeros(2 * n), jac=True, method="L-BFGS-B", bounds=[(0, None)] * (2 * n),
                   options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 5000})
    p_ref = ref.x[:n] - ref.x[n:]
    assert np.abs(r.x - p_ref).max() < 1e-4
    assert set(np.flatnonzero(np.abs(r.x) > 1e-8)) == set(np.flatnonzero(np.abs(p_ref) > 1e-6))


def test_two_phase_driver_on_oracle(oracle_case):
    """l1 phase with the Hoyer bisection, then the weighted l2 phase: the
    misfit drops by orders of magnitude, the two active Gaussians come out
    as the largest coefficients and k_f is recovered."""
    pr, p_true, d, obj = oracle_case
    cfg = inversion.InversionConfig(bisections=4, maxit_gist=60, opttol=1e-4, maxit_l2=100)
    res = inversion.invert(obj, pr.p.size, cfg)
    D0 = obj(np.zeros(pr.p.size), 0.05)[0]
    assert len(res.l1_betas) == 4 and all(0 <= h <= 1 for h in res.l1_hoyer)
    assert res.misfit < 1e-3 * D0
    assert set(np.argsort(-np.abs(res.p))[:2]) == {2, 5}   # the active Gaussians
    assert abs(res.p[2] - 0.8) < 0.05
    assert abs(res.k_f - 0.15) < 0.02
    assert res.grad_rel < 1e-4 or res.l2_iterations == cfg.maxit_l2


def test_more_thuente_backs_off_outside_the_domain():
    """phi = (s - 2)^2 - 4 is undefined past s = 3: started at s = 10 the
    search halves back into the domain and still meets the strong Wolfe
    conditions."""
    def phi(s):
        if s > 3.0:
            return math.inf, math.nan
        return (s - 2) ** 2 - 4, 2 * (s - 2)
    f0, g0 = phi(0.0)
    stp, f, g, nfev, info = optim.more_thuente(phi, f0, g0, stp=10.0, ftol=1e-4, gtol=0.5)
    assert info == "ok" and stp <= 3.0
    assert f <= f0 + 1e-4 * stp * g0 and abs(g) <= 0.5 * abs(g0)



def test_more_thuente_backs_off_across_a_pole():
    """phi = (s - 0.2)^2 + eps (1/s0 - 1/(s0 - s)) has a pole at s0 = 0.4:
    just past it the value is above phi(0) and the slope is negative and
    thousands of times steeper.  The search halves back below the pole and
    meets the strong Wolfe conditions there instead of interpolating
    across it."""
    s0, eps = 0.4, 1e-4

    def phi(s):
        return ((s - 0.2) ** 2 + eps * (1 / s0 - 1 / (s0 - s)),
                2 * (s - 0.2) - eps / (s0 - s) ** 2)
    f0, g0 = phi(0.0)
    f1, g1 = phi(0.4001)
    assert f1 > f0 and g1 < 1e3 * g0   # the guard's condition holds there
    stp, f, g, nfev, info = optim.more_thuente(phi, f0, g0, stp=0.4001, ftol=1e-4, gtol=0.9)
    assert info == "ok" and stp < s0 and nfev == 2
    assert f <= f0 + 1e-4 * stp * g0 and abs(g) <= 0.9 * abs(g0)
