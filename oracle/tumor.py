"""FP64 oracle of the tumor forward solve, its discrete adjoint, tangent and
Gauss-Newton Hessian products.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (Sec. 2.1, tumor forward operator and initial condition; coefficient
model with white matter only as in Sec. 4.1):
    dc/dt = div(k grad c) + rho c (1 - c),   k = k_f m,  rho = rho_f m,
    c(0) = Phi p = sum_i p_i Phi_i,  periodic on [0, 2 pi)^3.

Time discretization (Sec. 3.3): second-order Strang splitting with the
analytic solution of the logistic reaction and Crank-Nicolson for diffusion.
Reading taken (the paper does not print the splitting order): one step is
    a = R_{dt/2}(c^n);  (I - dt/2 A) b = (I + dt/2 A) a;  c^{n+1} = R_{dt/2}(b)
with A u = div(k grad u) and R_tau(u) = u E / (1 + u (E - 1)),
E = exp(rho tau), the exact flow of dc/dt = rho c (1 - c) over time tau.

Each Crank-Nicolson system is solved by preconditioned conjugate gradients
(scipy's routine as a library step) with the constant-coefficient Fourier
preconditioner (1 + dt/2 kbar |w|^2)^-1, kbar = k_f max(m), initial guess
x0 = a, stopped when ||r||_2 < rtol ||rhs||_2 (grid 2-norms).  The default
rtol = 1e-13 makes the result the exact solution of the discrete system up
to rounding.

Gradient: the paper derives the continuous adjoint and gradient with respect
to p (Phi^T alpha(0)) and k_f (time integral of m grad c . grad alpha), Sec.
2.1 optimality system, and evaluates it as state solve, adjoint solve,
gradient (Sec. 3.1).  This oracle instead differentiates the discrete map
exactly (discretize-then-optimize), so finite differences of the discrete
objective agree with it; it also returns the derivative with respect to
rho_f, which the paper does not invert.  The printed sign of the reaction
term in the continuous adjoint is not used; the discrete transpose fixes it.

Objective: J = 1/2 ||c(T) - d||^2_{L2} approximated by the periodic
trapezoid rule, J = 1/2 h^3 sum (c(T) - d)^2 (tumor misfit of Tab. 1).

Full coefficient and misfit model (Sec. 2.1): the diffusion and reaction
coefficients are tissue-weighted sums k = k_f sum_i k_i m_i and
rho = rho_f sum_i rho_i m_i over the WM/GM/CSF maps, so the diffusion field
m (``Setup.m``) and the reaction field (``Setup.m_rho``, default m) may
differ; the Gaussians are zero inside CSF, c(0) = w Phi p with a mask field
w (``Setup.phi_mask``, default 1; ``csf_mask`` gives w = 1 - m_CSF); and
the objective may add the anatomy-label misfit
D_m = 1/2 ||m (1 - c(T)) - m_P||^2 of the tumor-masked healthy labels
against the patient's (``misfit_labels``), whose derivative enters the
adjoint's terminal condition.

Parity pins: see tests/test_oracle_*.py (closed forms, invariants, dense 8^3
brute force with complex-step derivatives, finite differences).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse.linalg as spla

from . import spectral

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------- reaction
def reaction(u, m, rho_f, tau):
    """Exact logistic flow over time tau with rate rho = rho_f m."""
    E = np.exp(rho_f * m * tau)
    return u * E / (1.0 + u * (E - 1.0))


def reaction_du(u, m, rho_f, tau):
    """Derivative of the logistic flow with respect to its input u."""
    E = np.exp(rho_f * m * tau)
    D = 1.0 + u * (E - 1.0)
    return E / (D * D)


def reaction_drho(r_out, m, tau):
    """Derivative of the logistic flow with respect to rho_f, written in
    terms of its output R: dR/drho_f = m tau R (1 - R)."""
    return m * tau * r_out * (1.0 - r_out)


# ------------------------------------------------------------ Gaussian basis
def basis_factors(centres, sigma, n):
    """Per-axis factors g[i, a, j] = exp(-d(x_j, c_ia)^2 / (2 sigma^2)) with
    the minimum-image periodic distance d.  Phi_i(x) is their product
    (unnormalized Gaussians of standard deviation sigma, Sec. 4.1)."""
    x = np.arange(n) * (TWO_PI / n)
    c = np.asarray(centres, dtype=np.float64)
    d = np.abs(x[None, None, :] - c[:, :, None]) % TWO_PI
    d = np.minimum(d, TWO_PI - d)
    return np.exp(-d * d / (2.0 * sigma * sigma))


def phi(p, centres, sigma, n):
    """Initial condition c0 = Phi p = sum_i p_i Phi_i (Sec. 2.1)."""
    g = basis_factors(centres, sigma, n)
    out = np.zeros((n, n, n))
    for i, pi in enumerate(np.asarray(p, dtype=np.float64)):
        out += pi * (g[i, 0][:, None, None] * g[i, 1][None, :, None]
                     * g[i, 2][None, None, :])
    return out


def phi_t(field, centres, sigma):
    """Phi^T lam: (Phi^T lam)_i = sum_x Phi_i(x) lam(x) (plain grid sum)."""
    n = field.shape[0]
    g = basis_factors(centres, sigma, n)
    out = np.empty(len(g))
    for i in range(len(g)):
        out[i] = np.einsum("i,j,k,ijk->", g[i, 0], g[i, 1], g[i, 2], field)
    return out


# --------------------------------------------------------------- CN solves
@dataclasses.dataclass
class Setup:
    """Everything that stays fixed over one forward/adjoint evaluation."""
    m: np.ndarray
    centres: np.ndarray
    sigma: float
    rho_f: float
    k_f: float
    nt: int
    T: float = 1.0
    rtol: float = 1e-13
    maxit: int = 2000
    m_rho: np.ndarray | None = None     # reaction field (default: m)
    phi_mask: np.ndarray | None = None  # c(0) = phi_mask * Phi p (default 1)

    @property
    def n(self):
        return self.m.shape[0]

    @property
    def mr(self):
        """Field of the reaction coefficient rho = rho_f mr."""
        return self.m if self.m_rho is None else self.m_rho

    def masked(self, field):
        return field if self.phi_mask is None else self.phi_mask * field

    @property
    def dt(self):
        return self.T / self.nt

    @property
    def h3(self):
        return (TWO_PI / self.n) ** 3


def _cn_solve(setup: Setup, rhs, x0):
    """Solve (I - dt/2 k_f A_m) x = rhs by PCG; returns (x, iterations)."""
    n = setup.n
    shape = (n, n, n)
    k = setup.k_f * setup.m
    half = 0.5 * setup.dt
    sym = spectral.precond_symbol(n, setup.dt, setup.k_f * float(setup.m.max()))

    def mv(v):
        u = v.reshape(shape)
        return (u - half * spectral.diffusion(u, k)).ravel()

    def pc(v):
        return spectral.apply_precond(v.reshape(shape), sym).ravel()

    N3 = n ** 3
    op = spla.LinearOperator((N3, N3), matvec=mv, dtype=np.float64)
    M = spla.LinearOperator((N3, N3), matvec=pc, dtype=np.float64)
    its = [0]

    def cb(_):
        its[0] += 1

    x, info = spla.cg(op, rhs.ravel(), x0=x0.ravel().copy(), rtol=setup.rtol,
                      atol=0.0, maxiter=setup.maxit, M=M, callback=cb)
    if info != 0:
        raise RuntimeError(f"oracle CG did not reach rtol={setup.rtol} "
                           f"in {setup.maxit} iterations")
    return x.reshape(shape), its[0]


def _A_m(setup: Setup, u):
    """A_m u = div(m grad u), the diffusion operator per unit k_f."""
    return spectral.diffusion(u, setup.m)


# ----------------------------------------------------------------- forward
@dataclasses.dataclass
class Trajectory:
    c: list      # c^0 .. c^nt
    a: list      # a^n = R(c^n), n < nt
    b: list      # b^n, Crank-Nicolson output, n < nt
    its: list    # PCG iterations per step


def forward(setup: Setup, p) -> Trajectory:
    """State solve: Strang steps from c0 = Phi p (times the CSF mask, if
    set) to c(T)."""
    return forward_c0(setup, setup.masked(phi(p, setup.centres, setup.sigma, setup.n)))


def forward_c0(setup: Setup, c0) -> Trajectory:
    """State solve from a given initial field c0."""
    tau = 0.5 * setup.dt
    c = np.array(c0, dtype=np.float64, copy=True)
    tr = Trajectory([c], [], [], [])
    for _ in range(setup.nt):
        a = reaction(c, setup.mr, setup.rho_f, tau)
        rhs = a + tau * setup.k_f * _A_m(setup, a)
        b, its = _cn_solve(setup, rhs, a)
        c = reaction(b, setup.mr, setup.rho_f, tau)
        tr.a.append(a)
        tr.b.append(b)
        tr.c.append(c)
        tr.its.append(its)
    return tr


def misfit(setup: Setup, cT, d):
    """J = 1/2 h^3 sum (c(T) - d)^2 and its gradient h^3 (c(T) - d)."""
    r = cT - d
    return 0.5 * setup.h3 * float(np.sum(r * r)), setup.h3 * r


def misfit_labels(setup: Setup, cT, d, m_lab, m_pat):
    """J = D_c + D_m with D_m = 1/2 h^3 sum_x sum_i (m_i (1 - c) - mP_i)^2
    (Sec. 2.1 objective: the simulated tumor masks the healthy labels
    m_i, which are compared with the patient's labels mP_i), and its
    gradient in c(T):  h^3 [(c - d) - sum_i m_i (m_i (1 - c) - mP_i)].
    m_lab, m_pat: sequences of label fields."""
    J, lam = misfit(setup, cT, d)
    for mi, pi in zip(m_lab, m_pat):
        e = mi * (1.0 - cT) - pi
        J += 0.5 * setup.h3 * float(np.sum(e * e))
        lam = lam - setup.h3 * mi * e
    return J, lam


def coefficient_fields(tissues, k_w, rho_w):
    """Diffusion and reaction fields of the tissue-weighted coefficient
    model (Sec. 2.1): k = k_f sum_i k_i m_i, rho = rho_f sum_i rho_i m_i.
    Returns (sum_i k_i m_i, sum_i rho_i m_i)."""
    mk = sum(w * t for w, t in zip(k_w, tissues))
    mr = sum(w * t for w, t in zip(rho_w, tissues))
    return np.asarray(mk, dtype=np.float64), np.asarray(mr, dtype=np.float64)


def csf_mask(m_csf):
    """Mask of the initial condition: the Gaussians vanish where the
    tissue is CSF (Sec. 2.1); with a probability map, w = 1 - m_CSF."""
    return 1.0 - np.asarray(m_csf, dtype=np.float64)


# ----------------------------------------------------------------- adjoint
@dataclasses.dataclass
class Gradient:
    g_p: np.ndarray
    g_rho: float
    g_k: float
    lam0: np.ndarray     # cotangent with respect to c^0
    its: list
    g_mdiff: np.ndarray | None = None    # d/d m(x) of the diffusion field
    g_mreact: np.ndarray | None = None   # d/d mr(x) of the reaction field


def vjp(setup: Setup, tr: Trajectory, lamT, fields=False) -> Gradient:
    """Exact transpose of the discrete forward map applied to a cotangent
    lamT on c(T) (plain Euclidean pairing).  Returns d<lamT, c(T)>/d(p,
    rho_f, k_f) and the cotangent on c^0.

    fields=True also returns the derivatives with respect to the diffusion
    field m and the reaction field mr at every grid point: the discrete
    counterpart of the coupling field q(x) that the registration step of the
    Picard iteration receives (Sec. 2.2), a time integral of k_f grad c . grad(adjoint) and
    rho_f c (1 - c) (adjoint) terms.  Per step, with mu the Crank-Nicolson
    adjoint solution and s = a + b:
        g_mdiff  += -dt/2 k_f sum_j (D_j mu)(D_j s)   (D_j antisymmetric)
        g_mreact += rho_f dt/2 lam R (1 - R)          (each reaction half step)
    so that sum_x m g_mdiff = k_f g_k and sum_x mr g_mreact = rho_f g_rho."""
    tau = 0.5 * setup.dt
    m = setup.mr
    lam = np.array(lamT, dtype=np.float64, copy=True)
    g_rho = 0.0
    g_k = 0.0
    gmd = np.zeros_like(lam) if fields else None
    gmr = np.zeros_like(lam) if fields else None
    its = []
    for n in range(setup.nt - 1, -1, -1):
        cn, a, b, cn1 = tr.c[n], tr.a[n], tr.b[n], tr.c[n + 1]
        # c^{n+1} = R(b)
        g_rho += float(np.sum(lam * reaction_drho(cn1, m, tau)))
        if fields:
            gmr += setup.rho_f * lam * reaction_drho(cn1, 1.0, tau)
        lam = lam * reaction_du(b, m, setup.rho_f, tau)
        # (I - dt/2 A) b = (I + dt/2 A) a, A symmetric
        mu, it = _cn_solve(setup, lam, lam)
        its.append(it)
        Amu = _A_m(setup, mu)
        g_k += tau * float(np.sum(Amu * (a + b)))
        if fields:
            gmu, gs = spectral.grad(mu), spectral.grad(a + b)
            gmd -= tau * setup.k_f * sum(x * y for x, y in zip(gmu, gs))
        lam = mu + tau * setup.k_f * Amu
        # a = R(c^n)
        g_rho += float(np.sum(lam * reaction_drho(a, m, tau)))
        if fields:
            gmr += setup.rho_f * lam * reaction_drho(a, 1.0, tau)
        lam = lam * reaction_du(cn, m, setup.rho_f, tau)
    g_p = phi_t(setup.masked(lam), setup.centres, setup.sigma)
    return Gradient(g_p, g_rho, g_k, lam, its, gmd, gmr)


def gradient(setup: Setup, p, d, labels=None):
    """Reduced gradient of J (Sec. 3.1: state solve, adjoint solve,
    gradient).  labels = (m_lab, m_pat) adds the label misfit D_m.
    Returns (J, Gradient, Trajectory)."""
    tr = forward(setup, p)
    if labels is None:
        J, lamT = misfit(setup, tr.c[-1], d)
    else:
        J, lamT = misfit_labels(setup, tr.c[-1], d, *labels)
    return J, vjp(setup, tr, lamT), tr


# ------------------------------------------------------- tangent / GN HVP
def jvp(setup: Setup, tr: Trajectory, dc0, drho=0.0, dk=0.0):
    """Tangent of c(T) for a perturbation dc0 of c^0 and of rho_f, k_f."""
    tau = 0.5 * setup.dt
    m = setup.mr
    dc = np.array(dc0, dtype=np.float64, copy=True)
    for n in range(setup.nt):
        cn, a, b, cn1 = tr.c[n], tr.a[n], tr.b[n], tr.c[n + 1]
        da = reaction_du(cn, m, setup.rho_f, tau) * dc + reaction_drho(a, m, tau) * drho
        rhs = da + tau * setup.k_f * _A_m(setup, da) + tau * dk * _A_m(setup, a + b)
        db, _ = _cn_solve(setup, rhs, da)
        dc = reaction_du(b, m, setup.rho_f, tau) * db + reaction_drho(cn1, m, tau) * drho
    return dc


def gn_hvp(setup: Setup, tr: Trajectory, v):
    """Gauss-Newton Hessian-vector product for J with respect to p:
    H v = Phi^T J_c^T (h^3 I) J_c Phi v, about the trajectory ``tr``."""
    dc0 = setup.masked(phi(v, setup.centres, setup.sigma, setup.n))
    dcT = jvp(setup, tr, dc0)
    return vjp(setup, tr, setup.h3 * dcT).g_p
