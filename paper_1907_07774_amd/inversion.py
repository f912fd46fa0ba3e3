"""Tumor inversion driver on top of the GPU gradient (paper Sec. 2.3,
"Adaptivity and Convergence Criteria", and Sec. 3.1, "Regularization and
Nonlinear Solver Components for Tumor Inversion").

Two phases invert the Gaussian coefficients p and the diffusivity k_f of the
tumor model for fixed rho_f, healthy white matter m and observation d:

1. l1 phase: p only, k_f fixed (initially 0), objective D(p) + beta ||p||_1
   with D = 1/2 h^3 sum (c(T) - d)^2, solved by GIST (shrinkage steps with
   an Armijo-type step search).  beta is continued by bisection on the
   Hoyer sparsity measure H(p) = (n - ||p||_1/||p||_inf)/(n - 1): a solution
   with H above the target (0.95) asks for a smaller beta, one below it for
   a larger beta, starting from beta = ||grad D(p0)||_inf.
2. weighted-l2 phase: p and k_f, objective D(p, k_f) + beta_p/2 sum w_i
   p_i^2 with w_i = w_large where |p_i| < tau_S ||p^l1||_inf and w_small
   elsewhere, started from p^l1 and solved by L-BFGS with the Moré–Thuente
   line search until the gradient norm falls below opttol times the norm
   of the gradient at p = 0.

The paper alternates the two phases inside its outer (Picard) iteration,
each l1 phase holding k_f at the last l2 estimate; ``outer`` repeats the
pair that way without the registration step between them.

Every objective evaluation is one forward and one adjoint solve through the
C-ABI (``GpuMisfit``); the optimizer works on a few dozen float64 numbers on
the host.  Any callable with the same signature can stand in for the
objective.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import optim
from ._lib import TG_ERR_NOT_CONVERGED, TG_ERR_NUMERIC, TumorGradError


class GpuMisfit:
    """D(p, k_f) = 1/2 h^3 sum (c(T) - d)^2 and its gradient in (p, k_f),
    one forward + adjoint solve per call on a bound single-problem plan."""

    def __init__(self, plan, m, d, rho_f):
        import torch
        if plan.batch != 1:
            raise ValueError("GpuMisfit takes a single-problem plan")
        self.plan = plan
        dt = plan.dtype
        self.m = torch.as_tensor(m, dtype=dt, device=plan.device).contiguous()
        self.d = torch.as_tensor(d, dtype=dt, device=plan.device).contiguous()
        self.rho = torch.tensor([float(rho_f)], dtype=torch.float64, device=plan.device)
        self.evaluations = 0
        self.failures = 0

    def __call__(self, p, k_f):
        import torch
        dev = self.plan.device
        pt = torch.as_tensor(np.asarray(p, dtype=np.float64), device=dev)
        kt = torch.tensor([float(k_f)], dtype=torch.float64, device=dev)
        self.evaluations += 1
        try:
            self.plan.forward(pt, self.rho, kt, self.m)
            J, gp, _, gk = self.plan.adjoint_misfit(self.d)
        except TumorGradError as e:
            # a trial point where a solve broke down or went non-finite (e.g.
            # c^0 below the pole -1/(E-1) of the logistic step) is outside
            # the objective's domain: the line search backs off from it
            if e.status not in (TG_ERR_NOT_CONVERGED, TG_ERR_NUMERIC):
                raise
            self.failures += 1
            return math.inf, np.full(len(p), np.nan), math.nan
        return float(J), gp.cpu().numpy().astype(np.float64), float(gk)


@dataclass
class InversionConfig:
    """Solver settings.  beta_p and opttol follow the paper's table of
    parameters (1e-4, 1e-3); the phase-switch weights and threshold, the
    Hoyer target handling and the iteration caps are user settings the
    paper leaves open."""
    beta_p: float = 1e-4          # weighted-l2 regularization parameter
    opttol: float = 1e-3          # relative gradient tolerance of the l2 phase
    maxit_l2: int = 50            # L-BFGS iterations (the paper's Newton cap)
    tau_j: float = 1e-4           # GIST stopping tolerance
    maxit_gist: int = 100         # GIST iterations per beta
    hoyer_target: float = 0.95    # sparsity target of the beta continuation
    bisections: int = 6           # beta continuation steps
    tau_s: float = 0.1            # phase switch: small-coefficient threshold
    w_large: float = 1e2          # weight of the small coefficients
    w_small: float = 1.0          # weight of the others
    k_f0: float = 0.0             # k_f during the l1 phase
    k_f_init: float = 0.05        # k_f starting value of the l2 phase if k_f0 = 0
    k_f_min: float = 1e-4         # lower bound kept by the l2 line search
    k_scale: float = 0.1          # k_f is optimized as k_f / k_scale
    max_dp: float = 1.0           # largest change of any p_i in one l2 step
    skip_l1: bool = False         # start the l2 phase from p0 directly
    outer: int = 1                # l1 + l2 passes; each later l1 phase keeps
                                  # k_f at the previous l2 estimate


@dataclass
class InversionResult:
    p: np.ndarray
    k_f: float
    objective: float
    misfit: float
    grad_rel: float
    l1_betas: list = field(default_factory=list)
    l1_hoyer: list = field(default_factory=list)
    l1_iterations: int = 0
    l2_iterations: int = 0
    evaluations: int = 0
    converged: bool = False
    weights: np.ndarray | None = None


def l1_phase(obj, p0, k_f, cfg: InversionConfig):
    """GIST on D(p) + beta ||p||_1 for fixed k_f, with the Hoyer-driven
    bisection on beta.  Returns (p, betas, hoyer values, iterations, evals):
    the last solution that met the sparsity target (else the last nonzero
    one)."""
    fg = lambda p: obj(p, k_f)[:2]
    p = np.array(p0, dtype=np.float64)
    _, g0 = fg(p)
    # at p = 0, any beta >= ||grad D(0)||_inf keeps p = 0 optimal: the
    # search runs in (0, ||grad D||_inf)
    beta_lo, beta_hi = 0.0, float(np.abs(g0).max())
    beta = 0.5 * beta_hi
    best = None
    betas, hs = [], []
    its, nev = 0, 1
    for _ in range(cfg.bisections):
        r = optim.gist(fg, p, beta, tau_j=cfg.tau_j, maxit=cfg.maxit_gist)
        its += r.iterations
        nev += r.evaluations
        nonzero = float(np.abs(r.x).max()) > 0.0
        h = optim.hoyer(r.x) if nonzero else 1.0
        betas.append(beta)
        hs.append(h)
        if not nonzero:
            beta_hi = beta                  # everything shrunk away: smaller beta
        elif h >= cfg.hoyer_target:
            best, beta_hi = r.x, beta       # sparse enough: try a smaller beta
            p = r.x
        else:
            beta_lo = beta                  # too dense: larger beta
            p = r.x
        beta = 0.5 * (beta_lo + beta_hi)
    if best is None:
        best = p
    return best, betas, hs, its, nev


def l2_weights(p_l1, cfg: InversionConfig):
    pinf = float(np.abs(p_l1).max())
    return np.where(np.abs(p_l1) < cfg.tau_s * pinf, cfg.w_large, cfg.w_small)


def l2_phase(obj, p0, k0, w, g_ref_norm, cfg: InversionConfig):
    """L-BFGS + Moré–Thuente on D(p, k_f) + beta_p/2 sum w p^2 over
    (p, k_f / k_scale).  Returns the optimizer result and (p, k_f)."""
    n = p0.size
    ks = cfg.k_scale

    def fg(x):
        p, k = x[:n], x[n] * ks
        D, gp, gk = obj(p, k)
        f = D + 0.5 * cfg.beta_p * float((w * p) @ p)
        g = np.empty(n + 1)
        g[:n] = gp + cfg.beta_p * w * p
        g[n] = gk * ks
        return f, g

    def stpmax(x, d):
        # keep k_f >= k_f_min and move no p_i by more than max_dp: a long
        # step in p can push c^0 = Phi p past the logistic step's pole
        s = 1e20
        dp = float(np.abs(d[:n]).max())
        if dp > 0.0:
            s = cfg.max_dp / dp
        if d[n] < 0.0:
            s = min(s, max((x[n] - cfg.k_f_min / ks) / (-d[n]), 1e-12))
        return s

    x0 = np.concatenate([p0, [k0 / ks]])
    gref = np.zeros(n + 1)
    gref[0] = g_ref_norm
    r = optim.lbfgs(fg, x0, gtol_rel=cfg.opttol, g_ref=gref, maxit=cfg.maxit_l2,
                    stpmax_fn=stpmax)
    return r, r.x[:n].copy(), float(r.x[n] * ks)


def invert(obj, n_p, cfg: InversionConfig | None = None, p0=None) -> InversionResult:
    """Full two-phase inversion.  obj(p, k_f) -> (D, grad_p D, d D/d k_f)."""
    cfg = cfg or InversionConfig()
    p0 = np.zeros(n_p) if p0 is None else np.asarray(p0, dtype=np.float64)
    # reference gradient: the gradient at p = 0 (l2 phase stopping test)
    _, g_zero, _ = obj(np.zeros(n_p), cfg.k_f0 if cfg.k_f0 > 0 else cfg.k_f_init)
    g_ref = float(np.linalg.norm(g_zero))
    res = InversionResult(p=p0, k_f=cfg.k_f0, objective=np.nan, misfit=np.nan,
                          grad_rel=np.nan, evaluations=1)
    k_l1 = cfg.k_f0
    k0 = cfg.k_f0 if cfg.k_f0 > 0 else cfg.k_f_init
    for _ in range(max(1, cfg.outer)):
        if cfg.skip_l1:
            p_l1 = p0
            w = np.full(n_p, cfg.w_small)
        else:
            # every l1 phase starts from p0: its beta range comes from the
            # gradient there
            p_l1, betas, hs, its, nev = l1_phase(obj, p0, k_l1, cfg)
            res.l1_betas, res.l1_hoyer = betas, hs
            res.l1_iterations += its
            res.evaluations += nev
            w = l2_weights(p_l1, cfg)
        r, p, k = l2_phase(obj, p_l1, k0, w, g_ref, cfg)
        res.l2_iterations += r.iterations
        res.evaluations += r.evaluations
        k_l1 = k0 = k
    D = r.f - 0.5 * cfg.beta_p * float((w * p) @ p)
    res.p, res.k_f, res.objective, res.misfit = p, k, r.f, D
    res.grad_rel = float(np.linalg.norm(r.g)) / g_ref if g_ref > 0 else 0.0
    res.converged = r.converged
    res.weights = w
    return res
