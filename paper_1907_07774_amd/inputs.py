"""Seeded synthetic inputs for the tumor forward/adjoint path.

This module produces *data only*: white-matter phantoms, Gaussian-basis
centres and coefficients, growth parameters, Hessian directions and
observation masks.  It contains none of the method's arithmetic (no
reaction step, no basis evaluation, no diffusion operator), so both the
GPU path and the CPU oracle can read identical inputs from it.

Stand-ins for the paper's data (Sec. 4.1): the paper uses smoothed WM/GM/CSF
probability maps from 256^3 brain MRI, downsampled to 128^3, and grows the
tumor in white matter only.  Those images are not available, so a seeded
"brain-like" white-matter map is drawn instead: blobs inside an ellipsoid,
smoothed and clipped to [0, 1] (the idea of the SYN case of Sec. 4.4, an
elliptical WM region).  Gaussian basis centres sit on a regular g^3 grid
with spacing delta = 1.5 sigma around a seed point inside white matter
(Sec. 4.1, Tab. 2).

All draws use numpy's PCG64 ``default_rng(seed)`` in a fixed order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TWO_PI = 2.0 * math.pi

# Phantom geometry (domain [0, 2 pi)^3, periodic).
PHANTOM_CENTRE = (math.pi, math.pi, math.pi)
PHANTOM_AXES = (2.4, 2.0, 1.8)
PHANTOM_BLOBS = 12
PHANTOM_BLOB_SIGMA = (0.2, 0.6)
PHANTOM_SMOOTH = 0.1          # physical width of the spectral smoothing kernel

SIGMA_DEFAULT = TWO_PI / 30.0  # Gaussian basis width used in Sec. 4.1


def grid_coords(n: int) -> np.ndarray:
    """1D coordinates x_j = j h, h = 2 pi / n."""
    return np.arange(n, dtype=np.float64) * (TWO_PI / n)


def _periodic_delta(x: np.ndarray, c: float) -> np.ndarray:
    d = np.abs(x - c) % TWO_PI
    return np.minimum(d, TWO_PI - d)


@dataclasses.dataclass(frozen=True)
class PhantomSpec:
    blob_centres: np.ndarray   # (12, 3)
    blob_sigmas: np.ndarray    # (12,)


def phantom_spec(seed: int) -> PhantomSpec:
    """Blob parameters, independent of the grid so every resolution shows
    the same anatomy."""
    rng = np.random.default_rng(seed)
    centres = np.empty((PHANTOM_BLOBS, 3))
    sigmas = np.empty(PHANTOM_BLOBS)
    axes = np.asarray(PHANTOM_AXES)
    ctr = np.asarray(PHANTOM_CENTRE)
    for b in range(PHANTOM_BLOBS):
        while True:
            u = rng.uniform(-1.0, 1.0, size=3)
            if float(u @ u) <= 1.0:
                break
        centres[b] = ctr + axes * u
        sigmas[b] = rng.uniform(*PHANTOM_BLOB_SIGMA)
    return PhantomSpec(centres, sigmas)


def phantom(n: int, seed: int) -> np.ndarray:
    """White-matter probability map m(x) in [0, 1], shape (n, n, n), float64,
    C order with the last axis fastest."""
    spec = phantom_spec(seed)
    x = grid_coords(n)
    raw = np.zeros((n, n, n))
    for c, s in zip(spec.blob_centres, spec.blob_sigmas):
        gx = np.exp(-_periodic_delta(x, c[0]) ** 2 / (2 * s * s))
        gy = np.exp(-_periodic_delta(x, c[1]) ** 2 / (2 * s * s))
        gz = np.exp(-_periodic_delta(x, c[2]) ** 2 / (2 * s * s))
        raw += gx[:, None, None] * gy[None, :, None] * gz[None, None, :]
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    a = PHANTOM_AXES
    cc = PHANTOM_CENTRE
    inside = (((X - cc[0]) / a[0]) ** 2 + ((Y - cc[1]) / a[1]) ** 2
              + ((Z - cc[2]) / a[2]) ** 2) <= 1.0
    raw *= inside
    # Spectral Gaussian smoothing of fixed physical width (input preparation).
    kk = np.fft.fftfreq(n, 1.0 / n)
    kr = np.arange(n // 2 + 1, dtype=np.float64)
    w2 = (kk[:, None, None] ** 2 + kk[None, :, None] ** 2 + kr[None, None, :] ** 2)
    spec_f = np.fft.rfftn(raw) * np.exp(-0.5 * PHANTOM_SMOOTH ** 2 * w2)
    m = np.fft.irfftn(spec_f, s=(n, n, n), axes=(0, 1, 2))
    return np.clip(m, 0.0, 1.0)


def _smooth(raw: np.ndarray) -> np.ndarray:
    n = raw.shape[0]
    kk = np.fft.fftfreq(n, 1.0 / n)
    kr = np.arange(n // 2 + 1, dtype=np.float64)
    w2 = (kk[:, None, None] ** 2 + kk[None, :, None] ** 2 + kr[None, None, :] ** 2)
    spec_f = np.fft.rfftn(raw) * np.exp(-0.5 * PHANTOM_SMOOTH ** 2 * w2)
    return np.fft.irfftn(spec_f, s=(n, n, n), axes=(0, 1, 2))


def tissues(n: int, seed: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(WM, GM, CSF) probability maps, each (n, n, n) in [0, 1] with
    WM + GM + CSF <= 1: the white-matter phantom with two ventricles cut
    out, gray matter filling the rest of an ellipsoid 1.25x the
    white-matter one, CSF in the ventricles and in a rim around that
    ellipsoid (up to 1.4x); smoothed like the phantom.  The ventricle
    offsets are drawn with the seed."""
    wm = phantom(n, seed)
    rng = np.random.default_rng(20_000 + seed)
    x = grid_coords(n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    a = np.asarray(PHANTOM_AXES)
    cc = PHANTOM_CENTRE

    def ellipsoid(axes, centre):
        return ((((X - centre[0]) / axes[0]) ** 2 + ((Y - centre[1]) / axes[1]) ** 2
                 + ((Z - centre[2]) / axes[2]) ** 2) <= 1.0).astype(np.float64)
    vent = np.zeros((n, n, n))
    for side in (-1.0, 1.0):
        off = rng.uniform(-0.15, 0.15, size=3)
        ctr = (cc[0] + side * 0.45 + off[0], cc[1] + off[1], cc[2] + off[2])
        vent = np.maximum(vent, ellipsoid((0.3, 0.7, 0.35), ctr))
    brain = ellipsoid(1.25 * a, cc)
    rim = ellipsoid(1.4 * a, cc) - brain
    vent = np.clip(_smooth(vent), 0.0, 1.0)
    brain = np.clip(_smooth(brain), 0.0, 1.0)
    rim = np.clip(_smooth(rim), 0.0, 1.0)
    wm = wm * (1.0 - vent)
    csf = np.clip(vent + rim, 0.0, 1.0)
    gm = np.clip(brain - wm - vent, 0.0, 1.0)
    total = wm + gm + csf
    scale = np.where(total > 1.0, 1.0 / np.maximum(total, 1e-300), 1.0)
    return wm * scale, gm * scale, csf * scale


@dataclasses.dataclass(frozen=True)
class BasisSpec:
    centres: np.ndarray   # (n_p, 3) in [0, 2 pi)
    sigma: float
    p: np.ndarray         # (n_p,)


def basis(m: np.ndarray, g: int, seed: int, sigma: float = SIGMA_DEFAULT) -> BasisSpec:
    """g^3 Gaussian centres with spacing 1.5 sigma around a seed voxel drawn
    uniformly among voxels with m > 0.5, and coefficients p ~ U[0, 1]."""
    n = m.shape[0]
    rng = np.random.default_rng(seed)
    cand = np.flatnonzero(m.reshape(-1) > 0.5)
    if cand.size == 0:
        cand = np.array([int(np.argmax(m))])
    idx = int(cand[rng.integers(cand.size)])
    ix, iy, iz = np.unravel_index(idx, m.shape)
    h = TWO_PI / n
    seed_pt = np.array([ix * h, iy * h, iz * h])
    delta = 1.5 * sigma
    offs = np.arange(g, dtype=np.float64) - (g - 1) / 2.0
    cx, cy, cz = np.meshgrid(offs, offs, offs, indexing="ij")
    centres = seed_pt + delta * np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    centres = centres % TWO_PI
    p = rng.uniform(0.0, 1.0, size=g ** 3)
    return BasisSpec(centres, float(sigma), p)


def growth_params(seed: int) -> tuple[float, float]:
    """(rho_f, k_f) with rho_f ~ U[5, 15], k_f ~ U[0.01, 0.5]."""
    rng = np.random.default_rng(10_000 + seed)
    rho = float(rng.uniform(5.0, 15.0))
    kf = float(rng.uniform(0.01, 0.5))
    return rho, kf


def perturbed_p(p: np.ndarray, seed: int) -> np.ndarray:
    """p_obs = clip(p + 0.1 N(0, 1), 0, 1), drawn with seed + 1."""
    rng = np.random.default_rng(seed + 1)
    return np.clip(p + 0.1 * rng.standard_normal(p.shape), 0.0, 1.0)


def hvp_directions(ndir: int, n_p: int, seed: int) -> np.ndarray:
    """(ndir, n_p) directions, N(0, 1) entries, each row of unit length."""
    rng = np.random.default_rng(20_000 + seed)
    v = rng.standard_normal((ndir, n_p))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def random_field(n: int, seed: int, smooth: float = 0.3) -> np.ndarray:
    """A smooth zero-mean random field (test perturbations / cotangents)."""
    rng = np.random.default_rng(30_000 + seed)
    f = rng.standard_normal((n, n, n))
    kk = np.fft.fftfreq(n, 1.0 / n)
    kr = np.arange(n // 2 + 1, dtype=np.float64)
    w2 = (kk[:, None, None] ** 2 + kk[None, :, None] ** 2 + kr[None, None, :] ** 2)
    out = np.fft.irfftn(np.fft.rfftn(f) * np.exp(-0.5 * smooth ** 2 * w2), s=(n, n, n), axes=(0, 1, 2))
    return out / max(np.abs(out).max(), 1e-300)


def threshold_mask(c: np.ndarray, level: float = 0.5) -> np.ndarray:
    """Observation mask 1[c > level] (strict), as float64."""
    return (c > level).astype(np.float64)


@dataclasses.dataclass(frozen=True)
class Problem:
    n: int
    nt: int
    T: float
    m: np.ndarray
    centres: np.ndarray
    sigma: float
    p: np.ndarray
    rho_f: float
    k_f: float


def problem(n: int, g: int, seed: int, nt: int = 16, T: float = 1.0,
            rho_f: float | None = None, k_f: float | None = None,
            sigma: float = SIGMA_DEFAULT) -> Problem:
    """A full problem instance: phantom, basis, coefficients and parameters.
    If rho_f / k_f are not given they are drawn with ``growth_params``."""
    m = phantom(n, seed)
    b = basis(m, g, seed, sigma)
    r, k = growth_params(seed)
    return Problem(n, nt, T, m, b.centres, b.sigma, b.p,
                   r if rho_f is None else float(rho_f),
                   k if k_f is None else float(k_f))
