"""Fourier pseudo-spectral operators on the periodic grid [0, 2 pi)^3.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper discretizes space on a regular grid and takes derivatives with 3D
Fourier transforms under periodic boundary conditions (Sec. 2.1 notation and
boundary conditions; Sec. 3.3).  Readings taken where the paper is silent:

* First derivatives zero the Nyquist wavenumber (omega = -N/2), so each
  derivative D_j is a real antisymmetric matrix, the diffusion operator
  A = sum_j D_j k D_j is symmetric negative semidefinite and the
  Crank-Nicolson matrix I - dt/2 A is symmetric positive definite.
* FFTs are unnormalized forward and 1/N^3 inverse (numpy convention).

Parity unpinned by the paper itself (no worked example); pinned by closed
forms on trigonometric polynomials and by the dense 8^3 construction.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

# Transform library: numpy.fft by default; set_fft_workers(k) switches every
# transform of this module to scipy.fft (the same pocketfft algorithm) on k
# threads, for the large grids.  Results agree to rounding.
_WORKERS = None


def set_fft_workers(k):
    """k >= 1: scipy.fft with k threads; None: numpy.fft (the default)."""
    global _WORKERS
    _WORKERS = None if k is None else int(k)


def fft_workers():
    return _WORKERS


def rfftn(u):
    if _WORKERS is None:
        return np.fft.rfftn(u)
    return scipy.fft.rfftn(u, workers=_WORKERS)


def irfftn(uh, shape):
    if _WORKERS is None:
        return np.fft.irfftn(uh, s=shape, axes=(0, 1, 2))
    return scipy.fft.irfftn(uh, s=shape, axes=(0, 1, 2), workers=_WORKERS)


def wavenumbers(n: int):
    """Integer wavenumbers for a length-n periodic axis.

    Returns (w_full, w_half): w_full has numpy fftfreq order (0..n/2-1,
    -n/2..-1) and w_half is 0..n/2 for the halved last axis of a real
    transform.  The Nyquist entry (|w| = n/2) is set to zero in both, which
    is the derivative symbol used everywhere below.
    """
    w = np.fft.fftfreq(n, 1.0 / n)
    w[n // 2] = 0.0
    wh = np.arange(n // 2 + 1, dtype=np.float64)
    wh[n // 2] = 0.0
    return w, wh


def _symbols(n: int):
    w, wh = wavenumbers(n)
    return (w[:, None, None], w[None, :, None], wh[None, None, :])


def grad(u: np.ndarray) -> list[np.ndarray]:
    """Spectral gradient (D_x u, D_y u, D_z u), D_j u = F^-1(i w_j F u)."""
    n = u.shape[0]
    uh = rfftn(u)
    return [irfftn(1j * s * uh, u.shape) for s in _symbols(n)]


def div(v: list[np.ndarray]) -> np.ndarray:
    """Spectral divergence sum_j D_j v_j."""
    n = v[0].shape[0]
    out = None
    for s, vj in zip(_symbols(n), v):
        term = 1j * s * rfftn(vj)
        out = term if out is None else out + term
    return irfftn(out, v[0].shape)


def diffusion(u: np.ndarray, k: np.ndarray) -> np.ndarray:
    """A u = div(k grad u) with k a scalar field (isotropic diffusion,
    coefficient model of Sec. 2.1 with white matter only)."""
    g = grad(u)
    return div([k * gj for gj in g])


def precond_symbol(n: int, dt: float, kbar: float) -> np.ndarray:
    """Symbol of the constant-coefficient Fourier preconditioner
    (1 + dt/2 kbar |w|^2)^-1 on the half spectrum (Nyquist-zeroed w)."""
    sx, sy, sz = _symbols(n)
    return 1.0 / (1.0 + 0.5 * dt * kbar * (sx * sx + sy * sy + sz * sz))


def apply_precond(r: np.ndarray, sym: np.ndarray) -> np.ndarray:
    return irfftn(sym * rfftn(r), r.shape)
