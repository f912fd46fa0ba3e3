"""Registration transport on the GPU against the FP64 oracle, through
tg_transport / tg_transport_adjoint.

FP64: the same interpolation and spectral gradients in another order, so
the state and adjoint agree to rounding (1e-12) and the body force to
1e-10; FP32: 1e-5 relative.  At 128^3 and at the benchmark's 256^3, where
the whole-grid oracle is slow, the duality identity
<m(1), lam(1)> = <m(0), lam(0)> holds to the scheme's accuracy, and at
256^3 one step matches the oracle at sampled grid points.
"""
import math

import numpy as np
import pytest
import torch

from oracle import spectral, transport
from paper_1907_07774_amd import _lib, api, inputs

pytestmark = pytest.mark.gpu
TWO_PI = 2 * math.pi


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def grid(n):
    x = np.arange(n) * (TWO_PI / n)
    return np.meshgrid(x, x, x, indexing="ij")


def case(n, amp=0.6):
    """A compressible velocity (several cells per step at nt = 4), two label
    fields from the tissue phantom, a smooth terminal adjoint."""
    X, Y, Z = grid(n)
    v = [amp * np.sin(Y) + 0.3 * amp * np.cos(X), amp * np.cos(Z) + 0.2 * amp * np.sin(Y),
         amp * np.sin(X) - 0.25 * amp * np.cos(Z)]
    w = spectral.div(v)
    wm, gm, _ = inputs.tissues(n, 3)
    lam1 = [np.cos(X + Z), np.exp(0.5 * np.sin(Y))]
    return v, w, [wm, gm], lam1


def plan_for(n, precision):
    return api.Plan(n, 2, np.zeros((1, 3)), 0.3, precision=precision)


@pytest.mark.parametrize("n,nt", [(16, 4), (32, 3)])
def test_transport_and_adjoint_fp64(n, nt):
    print(f"case transport fp64 n={n} nt={nt}", flush=True)
    v, w, m0, lam1 = case(n)
    tr = transport.forward(v, m0, nt)
    lam0, b, _ = transport.adjoint(v, w, tr, lam1)
    plan = plan_for(n, "fp64")
    m1 = plan.transport(np.stack(v), np.stack(m0), nt, w=w).cpu().numpy()
    g0, gb = (x.cpu().numpy() for x in plan.transport_adjoint(np.stack(lam1)))
    for l in range(2):
        assert rel(m1[l], tr.m[-1][l]) < 1e-12
        assert rel(g0[l], lam0[l]) < 1e-12
    for j in range(3):
        assert rel(gb[j], b[j]) < 1e-10


def test_transport_divergence_free_fp64():
    """w = None: pure transport of the adjoint along -v."""
    print("case transport div-free fp64 n=16", flush=True)
    X, Y, Z = grid(16)
    v = [0.7 * np.sin(Y + Z), 0.5 * np.cos(Z + X), 0.6 * np.sin(X - Y)]   # div v = 0
    m0 = [np.exp(np.sin(X) * np.cos(Y))]
    lam1 = [np.cos(X + Z)]
    tr = transport.forward(v, m0, 4)
    lam0, b, _ = transport.adjoint(v, None, tr, lam1)
    plan = plan_for(16, "fp64")
    plan.transport(np.stack(v), np.stack(m0), 4)
    g0, gb = (x.cpu().numpy() for x in plan.transport_adjoint(np.stack(lam1)))
    assert rel(g0[0], lam0[0]) < 1e-12
    assert max(rel(gb[j], b[j]) for j in range(3)) < 1e-10


def test_transport_fp32_64():
    print("case transport fp32 n=64", flush=True)
    v, w, m0, lam1 = case(64)
    tr = transport.forward(v, m0, 4)
    lam0, b, _ = transport.adjoint(v, w, tr, lam1)
    plan = plan_for(64, "fp32")
    m1 = plan.transport(np.stack(v), np.stack(m0), 4, w=w).cpu().numpy()
    g0, gb = (x.cpu().numpy() for x in plan.transport_adjoint(np.stack(lam1)))
    assert max(rel(m1[l], tr.m[-1][l]) for l in range(2)) < 1e-5
    assert max(rel(g0[l], lam0[l]) for l in range(2)) < 1e-5
    assert max(rel(gb[j], b[j]) for j in range(3)) < 1e-5


def test_integer_shift_fp64():
    print("case transport integer shift", flush=True)
    n, nt = 32, 4
    h = TWO_PI / n
    shift = (2, -1, 3)
    v = np.stack([np.full((n,) * 3, s * h * nt) for s in shift])
    m0 = inputs.tissues(n, 5)[0][None]
    plan = plan_for(n, "fp64")
    m1 = plan.transport(v, m0, nt).cpu().numpy()[0]
    want = np.roll(m0[0], tuple(nt * s for s in shift), axis=(0, 1, 2))
    assert np.abs(m1 - want).max() < 1e-13


def test_transport_duality_128_fp32():
    """Three labels at 128^3 (FP32): the adjoint carries <m, lam> from t = 1
    back to t = 0 up to the scheme's error, and the plain tumor gradient
    of the same plan is unaffected by the transport calls in between."""
    print("case transport duality 128 fp32", flush=True)
    n = 128
    v, w, _, _ = case(n, 0.5)
    tis = np.stack(inputs.tissues(n, 7))
    X, Y, Z = grid(n)
    lam1 = np.stack([np.cos(X + Z), np.exp(0.5 * np.sin(Y)), np.sin(X) * np.cos(Z)])
    pr = inputs.problem(n, 2, 7, nt=4, rho_f=8.0, k_f=0.1)
    plan = api.Plan(n, 4, pr.centres, pr.sigma, rtol=1e-8, precision="fp32")
    cT = plan.forward(pr.p, pr.rho_f, pr.k_f, pr.m)
    g_before = plan.vjp(cT)[0].cpu().numpy()
    m1 = plan.transport(np.stack(v), tis, 8, w=w).double()
    lam0, _ = plan.transport_adjoint(lam1)
    a = float((m1 * torch.tensor(lam1, device=m1.device)).sum())
    b = float((torch.tensor(tis, device=m1.device) * lam0.double()).sum())
    assert abs(a - b) < 2e-3 * abs(a)
    g_after = plan.vjp(cT)[0].cpu().numpy()
    assert np.array_equal(g_before, g_after)
    del plan
    torch.cuda.empty_cache()


def test_transport_errors():
    print("case transport errors", flush=True)
    L = _lib.lib()
    plan = plan_for(16, "fp64")
    plan._bind()
    with pytest.raises(_lib.TumorGradError) as ei:
        plan.transport_adjoint(np.zeros((1, 16, 16, 16)))
    assert ei.value.status == _lib.TG_ERR_STATE
    v = torch.zeros(3 * 16 ** 3, dtype=torch.float64, device="cuda:0")
    m = torch.zeros(16 ** 3, dtype=torch.float64, device="cuda:0")
    small = torch.empty(1024, dtype=torch.uint8, device="cuda:0")
    st = L.tg_transport(plan._h, 2, 1, api._ptr(v), None, api._ptr(m), None,
                        api._ptr(small), 1024, None)
    assert st == _lib.TG_ERR_WORKSPACE
    assert L.tg_transport(plan._h, 0, 1, api._ptr(v), None, api._ptr(m), None,
                          api._ptr(small), 1024, None) == _lib.TG_ERR_ARG
    batch = api.Plan(16, 2, np.zeros((2, 1, 3)), 0.3, precision="fp64", batch=2)
    batch._bind()
    assert L.tg_transport(batch._h, 2, 1, api._ptr(v), None, api._ptr(m), None,
                          api._ptr(small), 1024, None) == _lib.TG_ERR_ARG


def test_zero_velocity_is_the_identity_fp64():
    """v = 0: every foot is the grid point itself, so the state and the
    adjoint are copied bit for bit and the body force is lam(1) grad m0
    (the trapezoid weights sum to 1)."""
    print("case transport zero velocity", flush=True)
    n = 32
    m0 = np.stack(inputs.tissues(n, 9)[:2])
    X, Y, Z = grid(n)
    lam1 = np.stack([np.cos(X + Z), np.sin(Y)])
    plan = plan_for(n, "fp64")
    m1 = plan.transport(np.zeros((3, n, n, n)), m0, 3).cpu().numpy()
    lam0, body = (x.cpu().numpy() for x in plan.transport_adjoint(lam1))
    assert np.array_equal(m1, m0) and np.array_equal(lam0, lam1)
    want = [sum(lam1[l] * spectral.grad(m0[l])[j] for l in range(2)) for j in range(3)]
    assert max(rel(body[j], want[j]) for j in range(3)) < 1e-12


def test_single_step_single_label_fp32():
    print("case transport one step one label", flush=True)
    v, w, m0, lam1 = case(32)
    tr = transport.forward(v, m0[:1], 1)
    lam0, b, _ = transport.adjoint(v, w, tr, lam1[:1])
    plan = plan_for(32, "fp32")
    m1 = plan.transport(np.stack(v), m0[0], 1, w=w).cpu().numpy()
    g0, gb = (x.cpu().numpy() for x in plan.transport_adjoint(lam1[0]))
    assert rel(m1[0], tr.m[-1][0]) < 1e-5 and rel(g0[0], lam0[0]) < 1e-5
    assert max(rel(gb[j], b[j]) for j in range(3)) < 1e-5


def bench_case_256():
    """The 256^3 transport workload of the benchmark (three tissue labels,
    velocity of up to about two cells per step at nt = 4), FP32-rounded
    so that the oracle sees the GPU's inputs."""
    n, nt = 256, 4
    X, Y, Z = grid(n)
    amp = 2.0 * nt * (TWO_PI / n) / 1.6
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    v = [f32(amp * (np.sin(Y) + 0.3 * np.cos(X))), f32(amp * (np.cos(Z) + 0.2 * np.sin(Y))),
         f32(amp * (np.sin(X) - 0.25 * np.cos(Z)))]
    w = f32(amp * (-0.3 * np.sin(X) + 0.2 * np.cos(Y) + 0.25 * np.sin(Z)))
    m0 = f32(np.stack(inputs.tissues(n, 0)))
    lam1 = f32(np.stack([np.cos(X + Z), np.exp(0.5 * np.sin(Y)), np.sin(X) * np.cos(Z)]))
    return v, w, m0, lam1


def test_transport_256_fp32_benchmark_configuration():
    """At the benchmark size and launch configuration: the duality identity
    over 4 steps, and one step of the state and of the adjoint at 512
    sampled grid points against the oracle's interpolation at the oracle's
    feet (the oracle evaluates single points)."""
    print("case transport 256 fp32 benchmark configuration", flush=True)
    n = 256
    v, w, m0, lam1 = bench_case_256()
    dev = torch.device("cuda:0")
    plan = plan_for(n, "fp32")
    m1 = plan.transport(np.stack(v), m0, 4, w=w).double()
    lam0, _ = plan.transport_adjoint(lam1)
    a = float((m1 * torch.tensor(lam1, device=dev)).sum())
    b = float((torch.tensor(m0, device=dev) * lam0.double()).sum())
    assert abs(a - b) < 2e-5 * abs(a)
    del m1, lam0
    rng = np.random.default_rng(256)
    idx = tuple(rng.integers(0, n, 512) for _ in range(3))
    m1 = plan.transport(np.stack(v), m0, 1, w=w).cpu().numpy()
    lam0, _ = (x.cpu().numpy() for x in plan.transport_adjoint(lam1))
    ys = transport.foot_at(v, 1.0, -1.0, idx)
    ya = transport.foot_at(v, 1.0, +1.0, idx)
    for l in range(3):
        want = transport.interpolate(m0[l], *ys)
        assert np.abs(m1[l][idx] - want).max() < 1e-5 * np.abs(m0[l]).max()
        src = lam1[l] * (1.0 + 0.5 * w)
        want = transport.interpolate(src, *ya) / (1.0 - 0.5 * w[idx])
        assert np.abs(lam0[l][idx] - want).max() < 1e-5 * np.abs(lam1[l]).max()
    del plan
    torch.cuda.empty_cache()


def test_zero_velocity_256_fp32():
    """v = 0 at 256^3: state and adjoint are copied bit for bit and the
    body force is lam(1) grad m0 (oracle spectral gradient)."""
    print("case transport zero velocity 256", flush=True)
    n = 256
    _, _, m0, lam1 = bench_case_256()
    plan = plan_for(n, "fp32")
    m1 = plan.transport(np.zeros((3, n, n, n), dtype=np.float32), m0[:1], 2).cpu().numpy()
    lam0, body = (x.cpu().numpy() for x in plan.transport_adjoint(lam1[:1]))
    assert np.array_equal(m1[0], m0[0].astype(np.float32))
    assert np.array_equal(lam0[0], lam1[0].astype(np.float32))
    g = spectral.grad(m0[0])
    assert max(rel(body[j], lam1[0] * g[j]) for j in range(3)) < 1e-5
    del plan
    torch.cuda.empty_cache()
