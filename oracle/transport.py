"""FP64 oracle of the registration transport: semi-Lagrangian advection of
the anatomy labels, its adjoint and the body force of the registration
gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).

State (Sec. 2.1, registration advection operator; registration state
equation of the optimality system): the labels are carried by a
stationary velocity v over the pseudo-time [0, 1],
    dm/dt + v . grad m = 0,   m(0) = m_A.
Adjoint (same system, registration adjoint equation, written for a
terminal value lam(1)):
    -dlam/dt - div(lam v) = 0,
which, with w = div v (the paper's constraint div v = w), is
-dlam/dt - v . grad lam - lam w = 0.  Gradient: the body force
    b(x) = integral_0^1 sum_l lam_l grad m_l dt,
whose projection enters the registration optimality condition; for
J = <lam1, m(1)> the derivative in v is -b (optimize-then-discretize, as
the paper does for the registration, Sec. 3.2).

Discretization (Sec. 3.3: unconditionally stable semi-Lagrangian time
stepping; spectral derivatives).  Readings taken where the paper defers to
its references:
  * characteristics by Heun's second-order Runge-Kutta step, the velocity
    interpolated at the predictor;
  * tricubic Lagrange interpolation on the periodic grid (4 nodes per axis,
    floor(p) - 1 .. floor(p) + 2);
  * the adjoint's source integrated by the trapezoid rule along the
    characteristic of -v;
  * the body force's time integral by the trapezoid rule over the nt + 1
    time levels, spectral gradients (Nyquist zeroed).
All steps are plain numpy; the interpolation sums its 64 terms explicitly.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import spectral

TWO_PI = 2.0 * math.pi


def lagrange_weights(t):
    """Cubic Lagrange weights of the nodes -1, 0, 1, 2 at offset t."""
    return ((-t * (t - 1.0) * (t - 2.0)) / 6.0,
            ((t + 1.0) * (t - 1.0) * (t - 2.0)) / 2.0,
            (-(t + 1.0) * t * (t - 2.0)) / 2.0,
            ((t + 1.0) * t * (t - 1.0)) / 6.0)


def interpolate(f, px, py, pz):
    """Tricubic Lagrange interpolation of the periodic grid field f at the
    points (px, py, pz), given in grid units (index space)."""
    n = f.shape[0]
    out = np.zeros(np.shape(px))
    base, wts = [], []
    for p in (px, py, pz):
        i0 = np.floor(p)
        base.append(i0.astype(np.int64))
        wts.append(lagrange_weights(p - i0))
    for a in range(4):
        ia = (base[0] + a - 1) % n
        for b in range(4):
            ib = (base[1] + b - 1) % n
            wab = wts[0][a] * wts[1][b]
            for c in range(4):
                ic = (base[2] + c - 1) % n
                out += wab * wts[2][c] * f[ia, ib, ic]
    return out


def grid_points(n):
    i = np.arange(n, dtype=np.float64)
    return np.meshgrid(i, i, i, indexing="ij")


def foot(v, dt, sign=-1.0):
    """Departure points (grid units) of the characteristics that reach the
    grid points after a step dt of the velocity sign * v (v: three
    physical-unit fields): Heun's step,
        X* = x + sign dt v(x),  X = x + sign dt/2 (v(x) + v(X*))."""
    return foot_at(v, dt, sign, grid_points(v[0].shape[0]))


def foot_at(v, dt, sign, idx):
    """The same departure points for the grid points idx = (i, j, k)
    (integer-valued arrays of any one shape)."""
    n = v[0].shape[0]
    h = TWO_PI / n
    X, Y, Z = (np.asarray(a, dtype=np.float64) for a in idx)
    at = tuple(np.asarray(a).astype(np.int64) for a in idx)
    vx = [vj[at] for vj in v]
    s = sign * dt / h
    Xs, Ys, Zs = X + s * vx[0], Y + s * vx[1], Z + s * vx[2]
    vs = [interpolate(vj, Xs, Ys, Zs) for vj in v]
    return (X + 0.5 * s * (vx[0] + vs[0]), Y + 0.5 * s * (vx[1] + vs[1]),
            Z + 0.5 * s * (vx[2] + vs[2]))


@dataclasses.dataclass
class Transport:
    m: list          # m[k][l]: label l at time level k = 0..nt
    feet_state: tuple
    feet_adj: tuple


def forward(v, m0, nt):
    """State: m^{k+1}(x) = m^k(X(x)), X the Heun foot of v over dt = 1/nt."""
    dt = 1.0 / nt
    Xf = foot(v, dt, -1.0)
    m = [[np.array(ml, dtype=np.float64) for ml in m0]]
    for _ in range(nt):
        m.append([interpolate(ml, *Xf) for ml in m[-1]])
    return Transport(m, Xf, foot(v, dt, +1.0))


def adjoint(v, w, tr: Transport, lam1):
    """Adjoint from lam(1) = lam1 backward: along the characteristics of -v,
        lam^k(x) (1 - dt/2 w(x)) = [lam^{k+1} (1 + dt/2 w)](Y(x)),
    and the body force b = sum_k c_k dt sum_l lam_l^k grad m_l^k
    (trapezoid weights c_0 = c_nt = 1/2).  w = div v (None: 0).
    Returns (lam^0 per label, b as three fields, lam per level)."""
    nt = len(tr.m) - 1
    dt = 1.0 / nt
    Y = tr.feet_adj
    lam = [np.array(l1, dtype=np.float64) for l1 in lam1]
    levels = [None] * (nt + 1)
    levels[nt] = lam
    for k in range(nt - 1, -1, -1):
        if w is None:
            lam = [interpolate(l, *Y) for l in lam]
        else:
            lam = [interpolate(l * (1.0 + 0.5 * dt * w), *Y) / (1.0 - 0.5 * dt * w)
                   for l in lam]
        levels[k] = lam
    b = [np.zeros_like(lam[0]) for _ in range(3)]
    for k in range(nt + 1):
        ck = 0.5 if k in (0, nt) else 1.0
        for ml, ll in zip(tr.m[k], levels[k]):
            g = spectral.grad(ml)
            for j in range(3):
                b[j] += ck * dt * ll * g[j]
    return lam, b, levels
