"""Pins of the registration-transport oracle against closed forms,
invariants and convergence orders (the scheme is optimize-then-discretize,
so its adjoint is pinned by the continuous identities it approximates)."""
import math

import numpy as np
import pytest

from oracle import spectral, transport

TWO_PI = 2 * math.pi


def grid(n):
    x = np.arange(n) * (TWO_PI / n)
    return np.meshgrid(x, x, x, indexing="ij")


def smooth(n, a=0.0):
    X, Y, Z = grid(n)
    return np.exp(0.5 * np.sin(X - a) + 0.3 * np.cos(2 * Y) + 0.4 * np.sin(Z + 1.0))


def test_lagrange_weights_partition_and_nodes():
    for t in (0.0, 0.25, 0.5, 0.9):
        w = transport.lagrange_weights(t)
        assert abs(sum(w) - 1.0) < 1e-15
        assert abs(sum(wi * x for wi, x in zip(w, (-1, 0, 1, 2))) - t) < 1e-15
    assert transport.lagrange_weights(0.0) == (0.0, 1.0, 0.0, 0.0)


def test_interpolation_reproduces_tricubics():
    """A polynomial of degree <= 3 in each index is reproduced exactly away
    from the periodic seam."""
    n = 16
    i = np.arange(n, dtype=np.float64)
    I, J, K = np.meshgrid(i, i, i, indexing="ij")
    f = (I / 8) ** 3 - 2 * (I / 8) * (J / 8) ** 2 + (K / 8) ** 3 * (J / 8) + 0.5 * (I * J * K) / 512
    rng = np.random.default_rng(1)
    p = rng.uniform(2.0, 12.0, (3, 200))
    got = transport.interpolate(f, *p)
    x, y, z = p / 8
    want = x ** 3 - 2 * x * y ** 2 + z ** 3 * y + 0.5 * x * y * z
    assert np.abs(got - want).max() < 1e-12


def test_integer_shift_is_exact():
    """A constant velocity moving whole cells per step: the transport is a
    periodic shift."""
    n, nt = 16, 4
    h = TWO_PI / n
    shift = (2, -1, 3)                  # cells per step
    v = [np.full((n,) * 3, s * h * nt) for s in shift]
    m0 = [smooth(n), smooth(n, 1.0)]
    tr = transport.forward(v, m0, nt)
    for l in range(2):
        want = np.roll(m0[l], tuple(nt * s for s in shift), axis=(0, 1, 2))
        assert np.abs(tr.m[-1][l] - want).max() < 1e-13


def test_translation_is_fourth_order_in_space():
    """Constant fractional velocity: the exact state is the translated
    field; the error falls like h^4 (interpolation) when the grid is
    refined at a fixed number of steps."""
    errs = []
    for n in (32, 64):
        v = [np.full((n,) * 3, c) for c in (0.37, -0.21, 0.13)]
        X, Y, Z = grid(n)
        m0 = [np.exp(0.5 * np.sin(X) + 0.3 * np.cos(2 * Y) + 0.4 * np.sin(Z + 1.0))]
        tr = transport.forward(v, m0, 4)
        want = np.exp(0.5 * np.sin(X - 0.37) + 0.3 * np.cos(2 * (Y + 0.21))
                      + 0.4 * np.sin(Z - 0.13 + 1.0))
        errs.append(np.abs(tr.m[-1][0] - want).max())
    assert 11.0 < errs[0] / errs[1] < 22.0, errs


def test_heun_foot_exact_for_shear():
    """v = (sin y, 0, 0): the characteristics are straight lines in x and
    Heun's step reproduces them exactly."""
    n, dt = 16, 0.3
    X, Y, Z = grid(n)
    v = [np.sin(Y), np.zeros_like(X), np.zeros_like(X)]
    fx, fy, fz = transport.foot(v, dt, -1.0)
    h = TWO_PI / n
    I, J, K = transport.grid_points(n)
    assert np.abs(fx - (I - dt * np.sin(Y) / h)).max() < 1e-12
    assert np.abs(fy - J).max() < 1e-14 and np.abs(fz - K).max() < 1e-14


def compressible_velocity(n, amp=0.6):
    X, Y, Z = grid(n)
    v = [amp * np.sin(Y) + 0.3 * amp * np.cos(X), amp * np.cos(Z) + 0.2 * amp * np.sin(Y),
         amp * np.sin(X) - 0.25 * amp * np.cos(Z)]
    return v, spectral.div(v)


def duality_gap(n, nt, with_source=True):
    v, w = compressible_velocity(n)
    X, Y, Z = grid(n)
    m0 = [np.exp(np.sin(X) * np.cos(Y)), np.cos(Z) * np.sin(X + Y)]
    lam1 = [np.cos(X + Z), np.exp(0.5 * np.sin(Y))]
    tr = transport.forward(v, m0, nt)
    lam0, _, _ = transport.adjoint(v, w if with_source else None, tr, lam1)
    a = sum(float(np.sum(mm * ll)) for mm, ll in zip(tr.m[-1], lam1))
    b = sum(float(np.sum(mm * ll)) for mm, ll in zip(m0, lam0))
    return abs(a - b) / abs(a)


def test_adjoint_duality_converges():
    """<m(1), lam(1)> = <m(0), lam(0)> for the transport and its adjoint
    -lam_t - div(lam v) = 0; the discrete gap shrinks under refinement in
    space and time (second order in dt), with a compressible v."""
    g1 = duality_gap(32, 8)
    g2 = duality_gap(64, 16)
    assert g1 < 3e-3 and g2 < g1 / 3.0, (g1, g2)


def test_mutation_dropped_adjoint_source_is_caught():
    assert duality_gap(32, 8, with_source=False) > 10 * duality_gap(32, 8)


def fd_check(n, nt, eps=1e-6):
    v, w = compressible_velocity(n, 0.4)
    X, Y, Z = grid(n)
    m0 = [np.exp(np.sin(X) * np.cos(Y))]
    lam1 = [np.cos(X + Z) + 0.3]
    rng = np.random.default_rng(7)
    dv = [np.cos(X + 2 * Y) * rng.uniform(0.5, 1.0), np.sin(Z - X), np.cos(Y) * np.sin(Z)]

    def J(vv):
        return float(np.sum(transport.forward(vv, m0, nt).m[-1][0] * lam1[0]))
    fd = (J([a + eps * d for a, d in zip(v, dv)]) - J([a - eps * d for a, d in zip(v, dv)])) / (2 * eps)
    tr = transport.forward(v, m0, nt)
    _, b, _ = transport.adjoint(v, w, tr, lam1)
    ad = -sum(float(np.sum(bj * dj)) for bj, dj in zip(b, dv))
    return abs(ad - fd) / abs(fd)


def test_body_force_gradient_matches_finite_differences():
    """dJ/dv = -b for J = <lam1, m(1)> (continuous identity; the discrete
    gradient of the discrete J differs from it at the scheme's order and
    the difference shrinks under refinement)."""
    e1 = fd_check(32, 8)
    e2 = fd_check(64, 16)
    assert e1 < 3e-2 and e2 < e1 / 2.5, (e1, e2)
