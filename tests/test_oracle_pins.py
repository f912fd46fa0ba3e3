"""Pins of the FP64 oracle against things other than itself.

Each test fixes one part of the oracle by a closed form, an invariant, an
independent library routine or a brute-force dense construction, so that a
plausible mistake (dropped term, wrong sign, wrong index, transposed
operand) fails at least one of them.  The mutation tests at the end plant
such mistakes in the oracle and check that a pin catches them.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import dense, spectral, tumor
from paper_1907_07774_amd import inputs

TWO_PI = 2 * math.pi


def grid(n):
    x = np.arange(n) * (TWO_PI / n)
    return np.meshgrid(x, x, x, indexing="ij")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# ------------------------------------------------------------ spectral ops
@pytest.mark.parametrize("w", [(1, 0, 0), (0, 3, 0), (0, 0, 5), (2, -3, 7), (-7, 7, -7)])
def test_derivative_closed_form(w):
    """D_j sin(w.x) = w_j cos(w.x) for |w_j| < n/2 (Sec. 3.3: derivatives by
    3D Fourier transforms)."""
    n = 16
    X, Y, Z = grid(n)
    ph = w[0] * X + w[1] * Y + w[2] * Z
    g = spectral.grad(np.sin(ph))
    for j in range(3):
        assert np.abs(g[j] - w[j] * np.cos(ph)).max() < 1e-12


def test_derivative_nyquist_zero():
    """Reading: the Nyquist mode has zero first derivative."""
    n = 8
    X, Y, Z = grid(n)
    for j, A in enumerate((X, Y, Z)):
        g = spectral.grad(np.cos(n // 2 * A))
        assert np.abs(g[j]).max() < 1e-13


@pytest.mark.parametrize("w", [(1, 2, 3), (0, 0, 7), (5, -1, 0)])
def test_diffusion_constant_k_closed_form(w):
    """div(k grad cos(w.x)) = -k |w|^2 cos(w.x) for constant k."""
    n = 16
    X, Y, Z = grid(n)
    u = np.cos(w[0] * X + w[1] * Y + w[2] * Z)
    k = 0.37 * np.ones_like(u)
    Au = spectral.diffusion(u, k)
    assert np.abs(Au + 0.37 * sum(c * c for c in w) * u).max() < 1e-12


def test_diffusion_variable_k_closed_form():
    """k = 1 + 0.5 cos(x), u = sin(x):  d/dx(k du/dx) = -sin(x) - 0.5 sin(2x)."""
    n = 16
    X, _, _ = grid(n)
    k = 1.0 + 0.5 * np.cos(X)
    Au = spectral.diffusion(np.sin(X), k)
    assert np.abs(Au - (-np.sin(X) - 0.5 * np.sin(2 * X))).max() < 1e-12


def test_spectral_matches_dense_8():
    """FFT-based A equals the dense DFT-matrix construction at 8^3."""
    n = 8
    m = inputs.phantom(n, 4)
    u = inputs.random_field(n, 2)
    Ds = dense.derivative_3d(n)
    A = dense.diffusion_matrix(m.ravel(), Ds)
    assert np.abs(A @ u.ravel() - spectral.diffusion(u, m).ravel()).max() < 1e-13
    for j in range(3):
        assert np.abs(Ds[j] @ u.ravel() - spectral.grad(u)[j].ravel()).max() < 1e-13


def test_diffusion_symmetric_negative_semidefinite():
    n = 16
    m = inputs.phantom(n, 1)
    u = inputs.random_field(n, 3)
    v = inputs.random_field(n, 4)
    Au, Av = spectral.diffusion(u, m), spectral.diffusion(v, m)
    assert abs(np.sum(Au * v) - np.sum(u * Av)) < 1e-12 * np.abs(Au).max() * n ** 3
    assert np.sum(Au * u) <= 0.0


# --------------------------------------------------------------- time steps
def setup_const(n, k_f, rho_f, nt, T=1.0, rtol=1e-14):
    m = np.ones((n, n, n))
    return tumor.Setup(m, np.zeros((1, 3)), 0.3, rho_f, k_f, nt, T, rtol=rtol)


@pytest.mark.parametrize("w", [(1, 0, 0), (2, 1, 3)])
def test_cn_single_mode_exact_discrete(w):
    """Constant k, rho = 0, c0 = cos(w.x): each Crank-Nicolson step multiplies
    the mode by g = (1 - z/2)/(1 + z/2), z = dt k |w|^2; the Fourier
    preconditioner is exact so PCG needs one iteration."""
    n, nt, kf = 16, 8, 0.05
    su = setup_const(n, kf, 0.0, nt)
    X, Y, Z = grid(n)
    c0 = np.cos(w[0] * X + w[1] * Y + w[2] * Z)
    tr = tumor.forward_c0(su, c0)
    z = su.dt * kf * sum(c * c for c in w)
    g = (1 - z / 2) / (1 + z / 2)
    assert np.abs(tr.c[-1] - g ** nt * c0).max() < 1e-13
    assert max(tr.its) <= 1


def test_cn_second_order_in_time():
    """Against the exact decay exp(-k |w|^2 T) the error falls by ~4 per
    halving of dt (second-order Crank-Nicolson / Strang, Sec. 3.3)."""
    n, kf, T = 16, 0.2, 1.0
    X, Y, Z = grid(n)
    w = (2, 1, 1)
    c0 = np.cos(2 * X + Y + Z)
    exact = math.exp(-kf * 6 * T) * c0
    errs = []
    for nt in (4, 8, 16, 32):
        tr = tumor.forward_c0(setup_const(n, kf, 0.0, nt, T), c0)
        errs.append(np.abs(tr.c[-1] - exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.8 < r < 4.2 for r in ratios), ratios


def test_reaction_matches_ode_integration():
    """k_f = 0: c(T) must solve dc/dt = rho_f m c (1 - c) pointwise
    (logistic reaction of Sec. 2.1); checked against an independent
    high-order ODE integration."""
    n, nt, rho = 8, 4, 10.0
    m = inputs.phantom(n, 0) * 0.9 + 0.05
    rng = np.random.default_rng(5)
    c0 = rng.uniform(0, 1, (n, n, n))
    su = tumor.Setup(m, np.zeros((1, 3)), 0.3, rho, 0.0, nt)
    cT = tumor.forward_c0(su, c0).c[-1]
    idx = rng.choice(n ** 3, 64, replace=False)
    mm, y0 = m.ravel()[idx], c0.ravel()[idx]
    sol = solve_ivp(lambda t, y: rho * mm * y * (1 - y), (0, 1), y0,
                    method="DOP853", rtol=1e-13, atol=1e-15)
    assert np.abs(sol.y[:, -1] - cT.ravel()[idx]).max() < 1e-10


def test_reaction_only_stays_in_unit_interval():
    n = 8
    m = inputs.phantom(n, 2)
    c0 = np.random.default_rng(1).uniform(0, 1, (n, n, n))
    su = tumor.Setup(m, np.zeros((1, 3)), 0.3, 15.0, 0.0, 16)
    tr = tumor.forward_c0(su, c0)
    for c in tr.c:
        assert c.min() >= 0.0 and c.max() <= 1.0


@pytest.mark.parametrize("rtol", [1e-6, 1e-13])
def test_mass_conserved_without_reaction(rtol):
    """rho = 0: the mean mode is untouched by diffusion and preconditioner,
    so sum c is conserved for any solver tolerance."""
    n = 16
    m = inputs.phantom(n, 3)
    pr = inputs.basis(m, 2, 3)
    su = tumor.Setup(m, pr.centres, pr.sigma, 0.0, 0.3, 8, rtol=rtol)
    tr = tumor.forward(su, pr.p)
    s0, sT = tr.c[0].sum(), tr.c[-1].sum()
    assert abs(sT - s0) <= 1e-13 * abs(s0)


def test_strang_second_order_coupled():
    """Reaction + diffusion: self-convergence of order 2 in dt."""
    n = 16
    pr = inputs.problem(n, 2, 7, nt=8, rho_f=4.0, k_f=0.2)
    def cT(nt):
        su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, nt, rtol=1e-13)
        return tumor.forward(su, pr.p * 0.4).c[-1]
    ref = cT(128)
    e = [np.abs(cT(nt) - ref).max() for nt in (8, 16, 32)]
    r = [e[0] / e[1], e[1] / e[2]]
    assert all(3.5 < x < 4.5 for x in r), r


def test_coupled_upper_bound_and_small_undershoot():
    """0 <= c <= 1 holds only up to a small Gibbs over/undershoot of the
    spectral discretization at the steep front where rho drops to zero at
    the white-matter edge (about 2e-2 below zero at 64^3, shrinking with
    resolution)."""
    n = 64
    pr = inputs.problem(n, 2, 0, nt=16, rho_f=10.0, k_f=0.1)
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, 16, rtol=1e-10)
    c0max = tumor.phi(pr.p, pr.centres, pr.sigma, n).max()
    tr = tumor.forward(su, pr.p / max(c0max, 1.0))
    assert tr.c[-1].max() <= 1.0
    assert tr.c[-1].min() >= -0.03


# ------------------------------------------------------ basis (IC) pinning
def test_phi_matches_dense_basis():
    n = 8
    m = inputs.phantom(n, 0)
    b = inputs.basis(m, 2, 0)
    Phi = dense.basis_matrix(b.centres, b.sigma, n)
    assert np.abs(Phi @ b.p - tumor.phi(b.p, b.centres, b.sigma, n).ravel()).max() < 1e-14
    lam = inputs.random_field(n, 1)
    assert np.abs(Phi.T @ lam.ravel() - tumor.phi_t(lam, b.centres, b.sigma)).max() < 1e-12


def test_phi_peak_is_one_at_centre():
    """Unnormalized Gaussians with peak value 1 at their centre."""
    n = 32
    h = TWO_PI / n
    c = np.array([[5 * h, 7 * h, 31 * h]])
    f = tumor.phi([1.0], c, 0.3, n)
    assert abs(f[5, 7, 31] - 1.0) < 1e-15
    assert abs(f[5, 7, 0] - math.exp(-h * h / (2 * 0.09))) < 1e-15  # periodic wrap


# ------------------------------------------------------- dense brute force
@pytest.fixture(scope="module")
def tiny():
    n, nt = 8, 4
    pr = inputs.problem(n, 2, 3, nt=nt, rho_f=10.0, k_f=0.1)
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, nt, rtol=1e-15)
    d = inputs.threshold_mask(tumor.forward(su, inputs.perturbed_p(pr.p, 3)).c[-1])
    return pr, su, d


def test_forward_matches_dense(tiny):
    pr, su, _ = tiny
    cs = dense.forward(pr.m, pr.centres, pr.sigma, pr.p, pr.rho_f, pr.k_f, pr.nt)
    tr = tumor.forward(su, pr.p)
    for n in range(pr.nt + 1):
        assert rel(tr.c[n], cs[n]) < 1e-12


def test_gradient_matches_dense_complex_step(tiny):
    """Whole discrete gradient (p, rho_f, k_f) against complex-step
    derivatives of the dense model."""
    pr, su, d = tiny
    J, g, _ = tumor.gradient(su, pr.p, d)
    gp, gr, gk = dense.complex_step_gradient(pr.m, pr.centres, pr.sigma, pr.p,
                                             pr.rho_f, pr.k_f, pr.nt, d)
    Jd = dense.objective(pr.m, pr.centres, pr.sigma, pr.p, pr.rho_f, pr.k_f, pr.nt, d)
    assert abs(J - Jd) < 1e-11 * abs(Jd)
    # The forward map amplifies rounding by up to prod(dR/du) ~ e^{rho T};
    # 1e-11 is far below any modelling error (a wrong term gives >= 1e-3).
    assert rel(g.g_p, gp) < 1e-11
    assert abs(g.g_rho - gr) < 1e-11 * abs(gr)
    assert abs(g.g_k - gk) < 1e-11 * abs(gk)


def test_gn_hvp_matches_dense(tiny):
    pr, su, _ = tiny
    tr = tumor.forward(su, pr.p)
    Jc = dense.jacobian_cT_c0(pr.m, pr.rho_f, pr.k_f, pr.nt,
                              [c.ravel() for c in tr.c])
    Phi = dense.basis_matrix(pr.centres, pr.sigma, pr.m.shape[0])
    H = su.h3 * (Jc @ Phi).T @ (Jc @ Phi)
    v = inputs.hvp_directions(2, Phi.shape[1], 0)
    for vi in v:
        assert rel(tumor.gn_hvp(su, tr, vi), H @ vi) < 1e-12


# ----------------------------------------------- adjoint identity, FD, HVP
@pytest.fixture(scope="module")
def small():
    n, nt = 16, 6
    pr = inputs.problem(n, 2, 11, nt=nt, rho_f=8.0, k_f=0.15)
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, nt, rtol=1e-14)
    tr = tumor.forward(su, pr.p)
    return pr, su, tr


def test_adjoint_identity(small):
    """<J x, y> = <x, J^T y> for the full-horizon linearization, including
    the rho_f and k_f directions."""
    pr, su, tr = small
    n = pr.m.shape[0]
    x = inputs.random_field(n, 5)
    y = inputs.random_field(n, 6)
    drho, dk = 0.7, -1.3
    lhs = float(np.sum(tumor.jvp(su, tr, x, drho, dk) * y))
    g = tumor.vjp(su, tr, y)
    rhs = float(np.sum(x * g.lam0)) + drho * g.g_rho + dk * g.g_k
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradient_central_fd(small):
    """Central finite differences, step 1e-6 max(1, |theta|), on the FP64
    discrete objective."""
    pr, su, _ = small
    d = inputs.threshold_mask(tumor.forward(su, inputs.perturbed_p(pr.p, 11)).c[-1])
    J, g, _ = tumor.gradient(su, pr.p, d)

    def Jat(p, rho, kf):
        s = tumor.Setup(pr.m, pr.centres, pr.sigma, rho, kf, su.nt, rtol=1e-14)
        return tumor.misfit(s, tumor.forward(s, p).c[-1], d)[0]

    h = 1e-6 * max(1.0, pr.rho_f)
    fd = (Jat(pr.p, pr.rho_f + h, pr.k_f) - Jat(pr.p, pr.rho_f - h, pr.k_f)) / (2 * h)
    assert abs(fd - g.g_rho) < 1e-6 * abs(g.g_rho)
    h = 1e-6
    fd = (Jat(pr.p, pr.rho_f, pr.k_f + h) - Jat(pr.p, pr.rho_f, pr.k_f - h)) / (2 * h)
    assert abs(fd - g.g_k) < 1e-6 * abs(g.g_k)
    u = inputs.hvp_directions(1, pr.p.size, 4)[0]
    fd = (Jat(pr.p + h * u, pr.rho_f, pr.k_f) - Jat(pr.p - h * u, pr.rho_f, pr.k_f)) / (2 * h)
    assert abs(fd - g.g_p @ u) < 1e-6 * np.linalg.norm(g.g_p)


def test_gn_hvp_symmetric_psd(small):
    pr, su, tr = small
    v, w = inputs.hvp_directions(2, pr.p.size, 9)
    Hv, Hw = tumor.gn_hvp(su, tr, v), tumor.gn_hvp(su, tr, w)
    assert abs(Hv @ w - v @ Hw) < 1e-12 * np.linalg.norm(Hv)
    assert v @ Hv > 0 and w @ Hw > 0


# ------------------------------------- full coefficient and misfit model
K_W, RHO_W = (1.0, 0.1, 0.0), (1.0, 0.3, 0.0)   # WM, GM, CSF weights


@pytest.fixture(scope="module")
def tiny_full():
    """8^3 with distinct diffusion and reaction fields from WM/GM/CSF maps,
    the CSF mask on Phi and the label misfit against another seed's
    tissues."""
    n, nt = 8, 4
    pr = inputs.problem(n, 2, 3, nt=nt, rho_f=10.0, k_f=0.1)
    tis = inputs.tissues(n, 3)
    pat = inputs.tissues(n, 4)
    mk, mr = tumor.coefficient_fields(tis, K_W, RHO_W)
    mask = tumor.csf_mask(tis[2])
    su = tumor.Setup(mk, pr.centres, pr.sigma, pr.rho_f, pr.k_f, nt, rtol=1e-15,
                     m_rho=mr, phi_mask=mask)
    d = inputs.threshold_mask(tumor.forward(su, inputs.perturbed_p(pr.p, 3)).c[-1])
    assert rel(mk, mr) > 0.1 and float(mask.min()) < 0.5   # the fields differ
    return pr, su, d, tis, pat


def test_coefficient_fields_are_weighted_sums():
    wm, gm, csf = inputs.tissues(8, 1)
    mk, mr = tumor.coefficient_fields((wm, gm, csf), (1.0, 0.5, 0.0), (0.0, 0.0, 2.0))
    assert np.array_equal(mk, wm + 0.5 * gm) and np.array_equal(mr, 2.0 * csf)


def test_full_model_forward_matches_dense(tiny_full):
    pr, su, _, _, _ = tiny_full
    cs = dense.forward(su.m, pr.centres, pr.sigma, pr.p, pr.rho_f, pr.k_f, pr.nt,
                       m_rho=su.m_rho, mask=su.phi_mask)
    tr = tumor.forward(su, pr.p)
    for k in range(pr.nt + 1):
        assert rel(tr.c[k], cs[k]) < 1e-12


def test_full_model_gradient_matches_dense_complex_step(tiny_full):
    """Gradient of D_c + D_m in (p, rho_f, k_f) with separate diffusion and
    reaction fields and the masked basis, against complex-step derivatives
    of the dense model."""
    pr, su, d, tis, pat = tiny_full
    J, g, _ = tumor.gradient(su, pr.p, d, labels=(tis, pat))
    kw = dict(m_rho=su.m_rho, mask=su.phi_mask, labels=(tis, pat))
    gp, gr, gk = dense.complex_step_gradient(su.m, pr.centres, pr.sigma, pr.p, pr.rho_f,
                                             pr.k_f, pr.nt, d, **kw)
    Jd = dense.objective(su.m, pr.centres, pr.sigma, pr.p, pr.rho_f, pr.k_f, pr.nt, d, **kw)
    assert abs(J - Jd) < 1e-11 * abs(Jd)
    assert rel(g.g_p, gp) < 1e-11
    assert abs(g.g_rho - gr) < 1e-11 * abs(gr)
    assert abs(g.g_k - gk) < 1e-11 * abs(gk)
    # the label term matters: without it the gradient is far off
    J0, g0, _ = tumor.gradient(su, pr.p, d)
    assert J - J0 > 1e-3 * J and rel(g0.g_p, gp) > 1e-3


def test_reaction_field_drives_the_reaction():
    """k_f = 0 with distinct fields: c(T) solves dc/dt = rho_f mr c (1 - c)
    from c0 = w Phi p pointwise (ODE integration), whatever the diffusion
    field is."""
    n, nt, rho = 8, 4, 10.0
    wm, gm, csf = inputs.tissues(n, 2)
    mk, mr = tumor.coefficient_fields((wm, gm, csf), (1.0, 0.0, 0.0), (0.3, 1.0, 0.1))
    mask = tumor.csf_mask(csf)
    rng = np.random.default_rng(6)
    cen = rng.uniform(0, TWO_PI, (5, 3))
    p = rng.uniform(0.2, 1.0, 5)
    su = tumor.Setup(mk, cen, 0.8, rho, 0.0, nt, m_rho=mr, phi_mask=mask)
    c0 = mask * tumor.phi(p, cen, 0.8, n)
    cT = tumor.forward(su, p).c[-1]
    idx = rng.choice(n ** 3, 64, replace=False)
    mm, y0 = mr.ravel()[idx], c0.ravel()[idx]
    sol = solve_ivp(lambda t, y: rho * mm * y * (1 - y), (0, 1), y0,
                    method="DOP853", rtol=1e-13, atol=1e-15)
    assert np.abs(sol.y[:, -1] - cT.ravel()[idx]).max() < 1e-10


def test_csf_mask_reduces_to_plain_basis_and_zeroes_csf():
    pr = inputs.problem(8, 2, 3, nt=2, rho_f=10.0, k_f=0.1)
    su1 = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, 2, phi_mask=np.ones((8,) * 3))
    su0 = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, 2)
    assert np.array_equal(tumor.forward(su1, pr.p).c[0], tumor.forward(su0, pr.p).c[0])
    csf = np.zeros((8,) * 3)
    csf[2:5, 1:6, 3:7] = 1.0
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, 2, phi_mask=tumor.csf_mask(csf))
    assert np.all(tumor.forward(su, pr.p).c[0][csf == 1.0] == 0.0)


# ------------------------------------------- coupling field q(x) = dJ/dm
def test_coupling_fields_match_dense_complex_step(tiny_full):
    """Derivatives of J (with the label misfit) with respect to the
    diffusion field m and the reaction field mr at every grid point,
    checked along random smooth directions and single grid points by
    complex-step derivatives of the dense model."""
    pr, su, d, tis, pat = tiny_full
    tr = tumor.forward(su, pr.p)
    _, lamT = tumor.misfit_labels(su, tr.c[-1], d, tis, pat)
    g = tumor.vjp(su, tr, lamT, fields=True)
    n = su.n
    h = 1e-30
    dirs = [inputs.random_field(n, 50), inputs.random_field(n, 51)]
    for idx in ((1, 2, 3), (4, 4, 4), (6, 1, 5)):
        e = np.zeros((n,) * 3)
        e[idx] = 1.0
        dirs.append(e)
    kw = dict(labels=(tis, pat), mask=su.phi_mask)
    for dm in dirs:
        Jd = dense.objective(su.m + 1j * h * dm, pr.centres, pr.sigma, pr.p, pr.rho_f, pr.k_f,
                             pr.nt, d, m_rho=su.m_rho, **kw)
        want = Jd.imag / h
        assert abs(float(np.sum(g.g_mdiff * dm)) - want) < 1e-10 * max(abs(want), 1e-12)
        Jr = dense.objective(su.m, pr.centres, pr.sigma, pr.p, pr.rho_f, pr.k_f, pr.nt, d,
                             m_rho=su.m_rho + 1j * h * dm, **kw)
        want = Jr.imag / h
        assert abs(float(np.sum(g.g_mreact * dm)) - want) < 1e-10 * max(abs(want), 1e-12)


def test_coupling_fields_scaling_identities(small):
    """Scaling the diffusion (reaction) field by 1 + eps scales k_f (rho_f):
    sum_x m g_mdiff = k_f g_k and sum_x mr g_mreact = rho_f g_rho."""
    pr, su, tr = small
    g = tumor.vjp(su, tr, inputs.random_field(su.n, 52), fields=True)
    assert abs(float(np.sum(su.m * g.g_mdiff)) - su.k_f * g.g_k) < 1e-12 * abs(su.k_f * g.g_k)
    assert abs(float(np.sum(su.mr * g.g_mreact)) - su.rho_f * g.g_rho) < \
        1e-12 * abs(su.rho_f * g.g_rho)


# ----------------------------------------------- mutations must be caught
def _mutant_gradient_error(monkeypatch, name, fn, tiny):
    pr, su, d = tiny
    monkeypatch.setattr(tumor, name, fn)
    J, g, _ = tumor.gradient(su, pr.p, d)
    gp, gr, gk = dense.complex_step_gradient(pr.m, pr.centres, pr.sigma, pr.p,
                                             pr.rho_f, pr.k_f, pr.nt, d)
    return max(rel(g.g_p, gp), abs(g.g_rho - gr) / abs(gr), abs(g.g_k - gk) / abs(gk))


def test_mutation_wrong_sign_drho_is_caught(monkeypatch, tiny):
    orig = tumor.reaction_drho
    err = _mutant_gradient_error(monkeypatch, "reaction_drho",
                                 lambda r, m, tau: -orig(r, m, tau), tiny)
    assert err > 1e-3


def test_mutation_dropped_diffusion_term_in_adjoint_is_caught(monkeypatch, tiny):
    orig = tumor._A_m
    calls = {"n": 0}

    def bad(setup, u):
        calls["n"] += 1
        return orig(setup, u) if calls["n"] <= setup.nt else 0.0 * u
    err = _mutant_gradient_error(monkeypatch, "_A_m", bad, tiny)
    assert err > 1e-3


def test_mutation_transposed_basis_axes_is_caught(monkeypatch, tiny):
    orig = tumor.basis_factors

    def bad(centres, sigma, n):
        g = orig(centres, sigma, n)
        return g[:, ::-1, :]
    pr, su, d = tiny
    monkeypatch.setattr(tumor, "basis_factors", bad)
    tr = tumor.forward(su, pr.p)
    cs = dense.forward(pr.m, pr.centres, pr.sigma, pr.p, pr.rho_f, pr.k_f, pr.nt)
    assert rel(tr.c[-1], cs[-1]) > 1e-3


def test_mutation_reaction_on_diffusion_field_is_caught(monkeypatch, tiny_full):
    """Using the diffusion field in the reaction (forgetting m_rho) breaks
    the dense match of the full model."""
    pr, su, _, _, _ = tiny_full
    bad = tumor.Setup(su.m, su.centres, su.sigma, su.rho_f, su.k_f, su.nt, rtol=su.rtol,
                      phi_mask=su.phi_mask)
    tr = tumor.forward(bad, pr.p)
    cs = dense.forward(su.m, pr.centres, pr.sigma, pr.p, pr.rho_f, pr.k_f, pr.nt,
                       m_rho=su.m_rho, mask=su.phi_mask)
    assert rel(tr.c[-1], cs[-1]) > 1e-3


def test_mutation_label_gradient_sign_is_caught(monkeypatch, tiny_full):
    """A wrong sign of the label term in the terminal cotangent fails the
    complex-step pin."""
    pr, su, d, tis, pat = tiny_full
    orig = tumor.misfit_labels

    def bad(setup, cT, dd, m_lab, m_pat):
        J, lam = orig(setup, cT, dd, m_lab, m_pat)
        J0, lam0 = tumor.misfit(setup, cT, dd)
        return J, lam0 - (lam - lam0)
    monkeypatch.setattr(tumor, "misfit_labels", bad)
    _, g, _ = tumor.gradient(su, pr.p, d, labels=(tis, pat))
    gp, _, _ = dense.complex_step_gradient(su.m, pr.centres, pr.sigma, pr.p, pr.rho_f, pr.k_f,
                                           pr.nt, d, m_rho=su.m_rho, mask=su.phi_mask,
                                           labels=(tis, pat))
    assert rel(g.g_p, gp) > 1e-3
