"""Small dense optimizers for the tumor inversion driver: a Moré–Thuente line
search, L-BFGS with it, and the GIST proximal-gradient iteration for an l1
penalty.  They act on a few dozen parameters (the Gaussian coefficients p
and k_f) and call back into an objective whose evaluation is one GPU
forward + adjoint solve, so they are plain host code on float64 vectors.

References (algorithms restated, not copied): J. J. Moré and D. J.
Thuente, "Line search algorithms with guaranteed sufficient decrease",
ACM TOMS 20 (1994); J. Nocedal and S. J. Wright, Numerical Optimization,
2nd ed., Alg. 7.4 (L-BFGS two-loop recursion); P. Gong et al., "A general
iterative shrinkage and thresholding algorithm for non-convex regularized
optimization problems", ICML 2013 (GIST).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------
# Moré–Thuente line search
def _trial_step(stx, fx, dx, sty, fy, dy, stp, fp, dp, brackt, stpmin, stpmax):
    """One safeguarded interpolation step of the Moré–Thuente method.

    (stx, fx, dx): best step so far, (sty, fy, dy): other end of the
    interval, (stp, fp, dp): current trial.  Returns the new interval ends,
    the bracketing flag and the next trial step.
    """
    sgnd = dp * (dx / abs(dx)) if dx != 0 else dp

    def cubic_min(a, fa, da, b, fb, db):
        # minimizer of the cubic interpolating (a, fa, da), (b, fb, db)
        theta = 3.0 * (fa - fb) / (b - a) + da + db
        s = max(abs(theta), abs(da), abs(db))
        gamma = s * math.sqrt(max(0.0, (theta / s) ** 2 - (da / s) * (db / s)))
        if b < a:
            gamma = -gamma
        p = (gamma - da) + theta
        q = ((gamma - da) + gamma) + db
        r = p / q
        return a + r * (b - a)

    if fp > fx:
        # case 1: higher function value; the minimum is bracketed
        stpc = cubic_min(stx, fx, dx, stp, fp, dp)
        stpq = stx + ((dx / ((fx - fp) / (stp - stx) + dx)) / 2.0) * (stp - stx)
        stpf = stpc if abs(stpc - stx) < abs(stpq - stx) else stpc + (stpq - stpc) / 2.0
        brackt = True
    elif sgnd < 0.0:
        # case 2: lower value, derivatives of opposite sign; bracketed
        stpc = cubic_min(stp, fp, dp, stx, fx, dx)
        stpq = stp + (dp / (dp - dx)) * (stx - stp)
        stpf = stpc if abs(stpc - stp) > abs(stpq - stp) else stpq
        brackt = True
    elif abs(dp) < abs(dx):
        # case 3: lower value, same-sign derivative that decreases in size
        theta = 3.0 * (fx - fp) / (stp - stx) + dx + dp
        s = max(abs(theta), abs(dx), abs(dp))
        gamma = s * math.sqrt(max(0.0, (theta / s) ** 2 - (dx / s) * (dp / s)))
        if stp > stx:
            gamma = -gamma
        p = (gamma - dp) + theta
        q = (gamma + (dx - dp)) + gamma
        r = p / q
        if r < 0.0 and gamma != 0.0:
            stpc = stp + r * (stx - stp)
        elif stp > stx:
            stpc = stpmax
        else:
            stpc = stpmin
        stpq = stp + (dp / (dp - dx)) * (stx - stp)
        if brackt:
            stpf = stpc if abs(stpc - stp) < abs(stpq - stp) else stpq
            bound = stp + 0.66 * (sty - stp)
            stpf = min(bound, stpf) if stp > stx else max(bound, stpf)
        else:
            stpf = stpc if abs(stpc - stp) > abs(stpq - stp) else stpq
            stpf = min(stpmax, max(stpmin, stpf))
    else:
        # case 4: lower value, same-sign derivative that does not decrease
        if brackt:
            stpf = cubic_min(stp, fp, dp, sty, fy, dy)
        else:
            stpf = stpmax if stp > stx else stpmin
    # update the interval of uncertainty
    if fp > fx:
        sty, fy, dy = stp, fp, dp
    else:
        if sgnd < 0.0:
            sty, fy, dy = stx, fx, dx
        stx, fx, dx = stp, fp, dp
    return stx, fx, dx, sty, fy, dy, brackt, stpf


def more_thuente(phi, f0, g0, stp=1.0, ftol=1e-4, gtol=0.9, xtol=1e-10,
                 stpmin=1e-20, stpmax=1e20, maxfev=30):
    """Step along a descent direction satisfying the strong Wolfe conditions
    phi(s) <= phi(0) + ftol s phi'(0) and |phi'(s)| <= gtol |phi'(0)|.

    phi(s) returns (value, derivative) along the direction.  Returns
    (step, value, derivative, evaluations, info) with info 'ok',
    'maxfev', 'xtol' or 'bounds' (then the best step found).

    A trial with a non-finite value or derivative, or one above phi(0)
    whose slope is negative and steeper than 1000 phi'(0), lies past a
    singularity of phi (the method assumes phi smooth): the upper bound
    drops to the midpoint between it and the best step, which is tried
    next; 'domain' is returned with the best step if maxfev runs out that
    way.
    """
    if g0 >= 0.0:
        raise ValueError("not a descent direction")
    stp = min(max(stp, stpmin), stpmax)
    brackt = False
    stage1 = True
    ftest_slope = ftol * g0
    width = stpmax - stpmin
    width1 = 2.0 * width
    stx, fx, gx = 0.0, f0, g0
    sty, fy, gy = 0.0, f0, g0
    smin, smax = 0.0, stp + 4.0 * stp
    nfev = 0
    while True:
        f, g = phi(stp)
        nfev += 1
        # a non-finite trial, or one above phi(0) whose slope is still
        # negative and a thousand times steeper than at 0, has a singularity
        # of phi between it and the best step; the cubic and quadratic models
        # are meaningless across it, so halve toward the best step instead
        if not (math.isfinite(f) and math.isfinite(g)) or (f > f0 and g < 1e3 * g0):
            if nfev >= maxfev:
                return stx, fx, gx, nfev, "domain"
            stp = stpmax = max(stx + 0.5 * (stp - stx), stpmin)
            continue
        ftest = f0 + stp * ftest_slope
        if f <= ftest and abs(g) <= gtol * (-g0):
            return stp, f, g, nfev, "ok"
        if nfev >= maxfev:
            return stp, f, g, nfev, "maxfev"
        if brackt and (stp <= smin or stp >= smax or smax - smin <= xtol * smax):
            return stp, f, g, nfev, "xtol"
        if stp == stpmax and f <= ftest and g <= ftest_slope:
            return stp, f, g, nfev, "bounds"
        if stp == stpmin and (f > ftest or g >= ftest_slope):
            return stp, f, g, nfev, "bounds"
        # stage 1 works on the auxiliary psi(s) = phi(s) - phi(0) - ftol s phi'(0)
        # until a step with psi <= 0 and phi' >= 0 is seen
        if stage1 and f <= ftest and g >= min(ftol, gtol) * g0:
            stage1 = False
        if stage1 and f <= fx and f > ftest:
            fm, fxm, fym = f - stp * ftest_slope, fx - stx * ftest_slope, fy - sty * ftest_slope
            gm, gxm, gym = g - ftest_slope, gx - ftest_slope, gy - ftest_slope
            stx, fxm, gxm, sty, fym, gym, brackt, stp_new = _trial_step(
                stx, fxm, gxm, sty, fym, gym, stp, fm, gm, brackt, smin, smax)
            fx, gx = fxm + stx * ftest_slope, gxm + ftest_slope
            fy, gy = fym + sty * ftest_slope, gym + ftest_slope
        else:
            stx, fx, gx, sty, fy, gy, brackt, stp_new = _trial_step(
                stx, fx, gx, sty, fy, gy, stp, f, g, brackt, smin, smax)
        # force sufficient shrinkage of the interval once bracketed
        if brackt:
            if abs(sty - stx) >= 0.66 * width1:
                stp_new = stx + 0.5 * (sty - stx)
            width1 = width
            width = abs(sty - stx)
            smin, smax = min(stx, sty), max(stx, sty)
        else:
            smin = stp_new + 1.1 * (stp_new - stx)
            smax = stp_new + 4.0 * (stp_new - stx)
        stp = min(max(stp_new, stpmin), stpmax)
        if (brackt and (stp <= smin or stp >= smax)) or (brackt and smax - smin <= xtol * smax):
            stp = stx


# --------------------------------------------------------------------------
# L-BFGS
@dataclass
class OptResult:
    x: np.ndarray
    f: float
    g: np.ndarray
    iterations: int
    evaluations: int
    converged: bool
    history: list = field(default_factory=list)


def lbfgs(fg, x0, gtol_rel=1e-6, g_ref=None, maxit=200, memory=10, stpmax_fn=None,
          callback=None):
    """Minimize f with gradient by L-BFGS (two-loop recursion) and the
    Moré–Thuente line search.

    fg(x) -> (f, g).  Stops when ||g|| <= gtol_rel ||g_ref|| (g_ref: the
    gradient at x0 unless given).  stpmax_fn(x, d), if given, bounds the
    step along d (e.g. to keep a parameter positive).
    """
    x = np.array(x0, dtype=np.float64)
    f, g = fg(x)
    nev = 1
    if not (math.isfinite(f) and np.all(np.isfinite(g))):
        raise ValueError("objective is not finite at the starting point")
    gref = np.linalg.norm(g if g_ref is None else g_ref)
    S, Y = [], []
    hist = [(f, float(np.linalg.norm(g)))]
    if gref == 0.0 or np.linalg.norm(g) <= gtol_rel * gref:
        return OptResult(x, f, g, 0, nev, True, hist)
    for it in range(1, maxit + 1):
        # two-loop recursion: d = -H g
        q = g.copy()
        alphas = []
        for s, y in reversed(list(zip(S, Y))):
            rho = 1.0 / float(y @ s)
            a = rho * float(s @ q)
            alphas.append((a, rho, s, y))
            q -= a * y
        if S:
            s, y = S[-1], Y[-1]
            q *= float(s @ y) / float(y @ y)
        else:
            q /= max(np.linalg.norm(g), 1e-300)  # first step: unit length
        for a, rho, s, y in reversed(alphas):
            b = rho * float(y @ q)
            q += (a - b) * s
        d = -q
        g0 = float(g @ d)
        if g0 >= 0.0:  # lost descent: restart from steepest descent
            S.clear()
            Y.clear()
            d = -g / max(np.linalg.norm(g), 1e-300)
            g0 = float(g @ d)
        stpmax = stpmax_fn(x, d) if stpmax_fn else 1e20

        seen = {}

        def phi(t):
            nonlocal nev
            ft, gt = fg(x + t * d)
            nev += 1
            seen[t] = gt
            return ft, float(gt @ d)

        stp, fn, _, _, info = more_thuente(phi, f, g0, stp=min(1.0, 0.99 * stpmax),
                                           stpmax=stpmax)
        if not fn < f:
            # no decrease along d (the search ended at its lower bound or on
            # noise): drop the curvature pairs and retry along steepest
            # descent; stop if that direction fails too
            if not S:
                break
            S.clear()
            Y.clear()
            continue
        xn = x + stp * d
        gn = seen[stp]
        s, y = xn - x, gn - g
        if float(s @ y) > 1e-12 * float(np.linalg.norm(s) * np.linalg.norm(y)):
            S.append(s)
            Y.append(y)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
        x, f, g = xn, fn, gn
        hist.append((f, float(np.linalg.norm(g))))
        if callback:
            callback(it, x, f, g)
        if np.linalg.norm(g) <= gtol_rel * gref:
            return OptResult(x, f, g, it, nev, True, hist)
    return OptResult(x, f, g, it, nev, False, hist)


# --------------------------------------------------------------------------
# GIST for D(p) + beta ||p||_1
def soft_threshold(v, t):
    return np.sign(v) * np.maximum(0.0, np.abs(v) - t)


def gist(fg, p0, beta, tau_j=1e-6, maxit=500, sigma=1e-5, alpha0=1.0, alpha_min=1e-30,
         alpha_max=1e30):
    """Proximal-gradient (shrinkage) iteration for D(p) + beta ||p||_1.

    Each step: p_sd = p - alpha grad D(p), p+ = sign(p_sd) max(0, |p_sd| -
    alpha beta); the step alpha starts from the Barzilai–Borwein value and
    is halved until F(p+) <= F(p) - sigma/(2 alpha) ||p+ - p||^2 (Armijo-type
    sufficient decrease).  Stops when |F(p+) - F(p)| < tau_j (1 + F(p0))
    and ||p+ - p||_inf < sqrt(tau_j) (1 + ||p+||_inf).
    """
    p = np.array(p0, dtype=np.float64)
    D, g = fg(p)
    nev = 1
    F = D + beta * float(np.abs(p).sum())
    F0 = F
    alpha = alpha0
    hist = [F]
    for it in range(1, maxit + 1):
        while True:
            pn = soft_threshold(p - alpha * g, alpha * beta)
            Dn, gn = fg(pn)
            nev += 1
            Fn = Dn + beta * float(np.abs(pn).sum())
            if Fn <= F - sigma / (2.0 * alpha) * float((pn - p) @ (pn - p)) or alpha <= alpha_min:
                break
            alpha *= 0.5
        s, y = pn - p, gn - g
        done = (abs(Fn - F) < tau_j * (1.0 + F0) and
                np.abs(s).max() < math.sqrt(tau_j) * (1.0 + np.abs(pn).max()))
        p, D, g, F = pn, Dn, gn, Fn
        hist.append(F)
        if done:
            return OptResult(p, F, g, it, nev, True, hist)
        sy = float(s @ y)
        alpha = float(s @ s) / sy if sy > 0 else alpha * 2.0
        alpha = min(max(alpha, alpha_min), alpha_max)
    return OptResult(p, F, g, maxit, nev, False, hist)


def hoyer(p):
    """Hoyer sparsity measure (n - ||p||_1/||p||_inf)/(n - 1) in [0, 1]."""
    n = p.size
    pinf = float(np.abs(p).max())
    if pinf == 0.0 or n < 2:
        return 1.0
    return (n - float(np.abs(p).sum()) / pinf) / (n - 1)
