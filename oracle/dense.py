"""Brute-force dense version of the discrete tumor model on tiny grids.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every operator is an explicit matrix: the 1D DFT matrix F[k, j] =
exp(-2 pi i k j / n) (not an FFT routine), the Nyquist-zeroed derivative
D1 = Re(F^-1 diag(i w) F), its Kronecker lifts to 3D, A = sum_j D_j diag(k)
D_j, and the Crank-Nicolson step S = (I - dt/2 A)^-1 (I + dt/2 A) by a dense
solve.  All functions accept complex parameters so that derivatives can be
taken by the complex-step method, which has no subtraction error.  This is
the "brute force on tiny inputs" pin of the FFT-based oracle.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def dft_matrix(n):
    j = np.arange(n)
    return np.exp(-2j * math.pi * np.outer(j, j) / n)


def derivative_matrix(n):
    """Real n x n matrix of the spectral first derivative with the Nyquist
    mode zeroed."""
    F = dft_matrix(n)
    Finv = np.conj(F) / n
    w = np.array([k if k < n // 2 else k - n for k in range(n)], dtype=np.float64)
    w[n // 2] = 0.0
    D = Finv @ np.diag(1j * w) @ F
    assert np.abs(D.imag).max() < 1e-12
    return D.real


def derivative_3d(n):
    D1 = derivative_matrix(n)
    I = np.eye(n)
    return [np.kron(np.kron(D1, I), I), np.kron(np.kron(I, D1), I),
            np.kron(np.kron(I, I), D1)]


def diffusion_matrix(k_flat, Ds):
    """A = sum_j D_j diag(k) D_j for a flattened coefficient field k."""
    return sum(D @ (k_flat[:, None] * D) for D in Ds)


def basis_matrix(centres, sigma, n):
    """Phi[x, i] = exp(-|x - c_i|^2_per / (2 sigma^2)), x flattened C-order."""
    x = np.arange(n) * (TWO_PI / n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    out = np.empty((n ** 3, len(centres)))
    for i, c in enumerate(np.asarray(centres)):
        d = np.abs(pts - c[None, :]) % TWO_PI
        d = np.minimum(d, TWO_PI - d)
        out[:, i] = np.exp(-np.sum(d * d, axis=1) / (2 * sigma * sigma))
    return out


def _R(u, m, rho, tau):
    E = np.exp(rho * m * tau)
    return u * E / (1.0 + u * (E - 1.0))


def forward(m, centres, sigma, p, rho_f, k_f, nt, T=1.0, m_rho=None, mask=None):
    """Dense Strang/Crank-Nicolson forward map; returns the list c^0..c^nt
    (flattened).  Parameters may be complex (complex-step).  m drives the
    diffusion, m_rho (default m) the reaction; c^0 = diag(mask) Phi p."""
    n = m.shape[0]
    mf = m.ravel()
    mr = mf if m_rho is None else m_rho.ravel()
    Ds = derivative_3d(n)
    dt = T / nt
    tau = 0.5 * dt
    A = k_f * diffusion_matrix(mf, Ds)
    I = np.eye(n ** 3)
    L = I - tau * A
    Rm = I + tau * A
    Phi = basis_matrix(centres, sigma, n)
    if mask is not None:
        Phi = mask.ravel()[:, None] * Phi
    c = Phi @ np.asarray(p)
    cs = [c]
    for _ in range(nt):
        a = _R(c, mr, rho_f, tau)
        b = np.linalg.solve(L, Rm @ a)
        c = _R(b, mr, rho_f, tau)
        cs.append(c)
    return cs


def objective(m, centres, sigma, p, rho_f, k_f, nt, d, T=1.0, m_rho=None, mask=None,
              labels=None):
    """J = 1/2 h^3 sum (c(T) - d)^2, plus 1/2 h^3 sum_i sum (m_i (1 - c(T))
    - mP_i)^2 if labels = (m_lab, m_pat) is given (written without abs so
    it stays analytic for complex-step)."""
    n = m.shape[0]
    h3 = (TWO_PI / n) ** 3
    c = forward(m, centres, sigma, p, rho_f, k_f, nt, T, m_rho, mask)[-1]
    r = c - d.ravel()
    J = 0.5 * h3 * np.sum(r * r)
    if labels is not None:
        for mi, pi in zip(*labels):
            e = mi.ravel() * (1.0 - c) - pi.ravel()
            J = J + 0.5 * h3 * np.sum(e * e)
    return J


def complex_step_gradient(m, centres, sigma, p, rho_f, k_f, nt, d, T=1.0, h=1e-30,
                          m_rho=None, mask=None, labels=None):
    """Gradient of J with respect to (p, rho_f, k_f) by the complex-step
    method: dJ/dx = Im J(x + i h e) / h."""
    kw = dict(m_rho=m_rho, mask=mask, labels=labels)
    p = np.asarray(p, dtype=np.float64)
    gp = np.empty_like(p)
    for i in range(p.size):
        pp = p.astype(np.complex128)
        pp[i] += 1j * h
        gp[i] = objective(m, centres, sigma, pp, rho_f, k_f, nt, d, T, **kw).imag / h
    g_rho = objective(m, centres, sigma, p, rho_f + 1j * h, k_f, nt, d, T, **kw).imag / h
    g_k = objective(m, centres, sigma, p, rho_f, k_f + 1j * h, nt, d, T, **kw).imag / h
    return gp, float(g_rho), float(g_k)


def jacobian_cT_c0(m, rho_f, k_f, nt, c_traj, T=1.0):
    """Dense Jacobian d c(T) / d c^0 along a trajectory (real inputs)."""
    n = m.shape[0]
    mf = m.ravel()
    Ds = derivative_3d(n)
    dt = T / nt
    tau = 0.5 * dt
    A = k_f * diffusion_matrix(mf, Ds)
    I = np.eye(n ** 3)
    S = np.linalg.solve(I - tau * A, I + tau * A)
    Jm = I
    for c in c_traj[:-1]:
        E = np.exp(rho_f * mf * tau)
        a = _R(c, mf, rho_f, tau)
        b = S @ a
        dRc = E / (1.0 + c * (E - 1.0)) ** 2
        dRb = E / (1.0 + b * (E - 1.0)) ** 2
        Jm = (dRb[:, None] * (S @ (dRc[:, None] * Jm)))
    return Jm
