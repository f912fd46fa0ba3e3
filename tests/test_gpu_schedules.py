"""Every launch schedule computes the same thing: plan-wide tile shapes and
per-pass overrides change only the summation order of the FP64 partial
sums, so forward states and gradients agree with the default schedule to
the solver tolerance (FP64, rtol 1e-12: 1e-9 relative), and with the
oracle at 32^3."""
import numpy as np
import pytest
import torch

from oracle import tumor
from paper_1907_07774_amd import _lib, api, inputs

pytestmark = pytest.mark.gpu

PLAN_WIDE = [(8, 1, 1, 1), (32, 2, 2, 4), (16, 4, 4, 1), (16, 8, 1, 4), (32, 1, 8, 1),
             (64, 2, 1, 1)]
PER_PASS = [
    ((16, 1, 2, 1), {"x_inv_grad": (8, 4), "y_inv_grad": (32, 1), "z_matvec": (8, 4),
                     "y_fwd_div": (16, 4), "x_fwd_div": (32, 1)}),
    ((32, 2, 1, 4), {"x_inv_grad": (32, 4), "y_inv_grad": (8, 1), "z_matvec": (16, 1),
                     "y_fwd_div": (64, 1), "x_fwd_div": (64, 4)}),
]


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problem(n):
    pr = inputs.problem(n, 2 if n <= 64 else 4, 5, nt=4, rho_f=8.0, k_f=0.15)
    mx = tumor.phi(pr.p, pr.centres, pr.sigma, n).max()
    return pr, pr.p / max(mx, 1.0)


def run(pr, p, d, schedule, passes=None, precision="fp64"):
    plan = api.Plan(pr.n, pr.nt, pr.centres, pr.sigma, rtol=1e-12, precision=precision,
                    schedule=schedule, passes=passes)
    cT = plan.forward(p, pr.rho_f, pr.k_f, pr.m).cpu().numpy()
    J, gp, gr, gk = plan.adjoint_misfit(d)
    got = {k: plan.get_pass(k) for k in api.Plan.KERNELS}
    out = (cT, float(J), gp.cpu().numpy(), float(gr), float(gk), plan.get_schedule(), got)
    del plan
    torch.cuda.empty_cache()
    return out


@pytest.fixture(scope="module", params=[32, 128])
def reference(request):
    n = request.param
    pr, p = problem(n)
    d = inputs.threshold_mask(tumor.forward(
        tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, pr.nt, rtol=1e-12),
        inputs.perturbed_p(p, 5)).c[-1])
    return pr, p, d, run(pr, p, d, (0, 0, 0, 0))


def check(a, b):
    assert rel(a[0], b[0]) < 1e-9
    assert abs(a[1] - b[1]) < 1e-9 * abs(b[1])
    assert rel(a[2], b[2]) < 1e-9
    assert abs(a[3] - b[3]) < 1e-9 * abs(b[3])
    assert abs(a[4] - b[4]) < 1e-9 * abs(b[4])


def test_default_schedule_matches_oracle(reference):
    pr, p, d, ref = reference
    if pr.n != 32:
        pytest.skip("oracle gradient checked at 32^3")
    print("case schedules oracle n=32", flush=True)
    su = tumor.Setup(pr.m, pr.centres, pr.sigma, pr.rho_f, pr.k_f, pr.nt, rtol=1e-13)
    J, g, tr = tumor.gradient(su, p, d)
    assert rel(ref[0], tr.c[-1]) < 1e-10
    assert rel(ref[2], g.g_p) < 1e-9


@pytest.mark.parametrize("sched", PLAN_WIDE)
def test_plan_wide_schedules_agree(reference, sched):
    pr, p, d, ref = reference
    print(f"case schedule n={pr.n} {sched}", flush=True)
    out = run(pr, p, d, sched)
    assert out[5] == sched
    check(out, ref)


@pytest.mark.parametrize("sched,passes", PER_PASS)
def test_per_pass_schedules_agree(reference, sched, passes):
    pr, p, d, ref = reference
    print(f"case per-pass schedule n={pr.n} {sched} {passes}", flush=True)
    out = run(pr, p, d, sched, passes)
    assert out[6] == passes
    check(out, ref)


def test_per_pass_fp32_agrees():
    print("case per-pass fp32 n=64", flush=True)
    pr, p = problem(64)
    plan_a = api.Plan(64, pr.nt, pr.centres, pr.sigma, rtol=1e-8, precision="fp32",
                      schedule=(16, 1, 1, 1))
    a = plan_a.forward(p, pr.rho_f, pr.k_f, pr.m).cpu().numpy()
    plan_b = api.Plan(64, pr.nt, pr.centres, pr.sigma, rtol=1e-8, precision="fp32",
                      schedule=(16, 1, 1, 1), passes=PER_PASS[0][1])
    b = plan_b.forward(p, pr.rho_f, pr.k_f, pr.m).cpu().numpy()
    assert rel(a, b) < 1e-5


def test_kernel_timer_samples_solves():
    """The kernel timer with every = k times the launches of one
    Crank-Nicolson solve in k (the first, then every k-th) and counts only
    their work: fewer timed launches, the same time per launch that did
    work, and every < 1 is an argument error."""
    print("case kernel timer sampling n=32", flush=True)
    pr, p = problem(32)
    nt = 8
    plan = api.Plan(32, nt, pr.centres, pr.sigma, rtol=1e-10, precision="fp64")
    plan.forward(p, pr.rho_f, pr.k_f, pr.m)
    out = {}
    for every in (1, 4, 100):
        plan.kernel_timer("z_matvec", every)
        plan.forward(p, pr.rho_f, pr.k_f, pr.m)
        out[every] = plan.kernel_timer_read()
    plan.kernel_timer(None)
    ms1, n1, b1 = out[1]
    ms4, n4, b4 = out[4]
    ms100, n100, b100 = out[100]
    assert n1 > n4 > 0 and b1 > b4 > 0
    # every 4th of the nt forward solves (and the right-hand-side matvecs of
    # those solves), so between a sixth and a half of the launches
    assert n1 / 6 < n4 < n1 / 2
    assert 0 < n100 < n4  # only the first solve
    with pytest.raises(_lib.TumorGradError):
        plan.kernel_timer("z_matvec", 0)


def test_schedule_errors():
    print("case schedule errors", flush=True)
    pr, p = problem(32)
    plan = api.Plan(32, pr.nt, pr.centres, pr.sigma, precision="fp64", schedule=(16, 1, 1, 1))
    for bad in [("z_matvec", 32, 1), ("x_inv_grad", 12, 1), ("x_fwd_div", 16, 2),
                ("y_fwd_div", 0, 1)]:
        with pytest.raises(_lib.TumorGradError) as e:
            plan.set_pass(*bad)
        assert e.value.status == _lib.TG_ERR_ARG
    assert _lib.lib().tg_plan_set_pass(plan._h, 6, 16, 1) == _lib.TG_ERR_ARG
    assert _lib.lib().tg_plan_set_pass(plan._h, 0, 16, 1) == _lib.TG_ERR_ARG
    # a rejected value leaves the schedule as it was
    assert plan.get_pass("x_inv_grad") == (16, 1)
    plan.set_pass("x_inv_grad", 8, 4)
    assert plan.get_pass("x_inv_grad") == (8, 4)
    assert plan.get_pass("z_matvec") == (8, 1)  # FP64 default: one complex per access
    plan.set_pass("z_matvec", 8, 4)
    assert plan.get_pass("z_matvec") == (8, 4)
    plan.set_schedule(32, 8, 1, 1)  # resets every pass
    assert plan.get_pass("x_inv_grad") == (32, 1)
    assert plan.get_pass("z_matvec") == (8, 1)
    with pytest.raises(_lib.TumorGradError):
        plan.set_pass("z_matvec", 0, 4)  # the wide z matvec has no per-pass variant
    plan.set_pass("z_matvec", *plan.get_pass("z_matvec"))  # its own shape: a no-op
    assert plan.get_pass("z_matvec") == (8, 1)
