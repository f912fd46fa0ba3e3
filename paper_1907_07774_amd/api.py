"""Python binding of libtumorgrad: plans, forward / gradient / Hessian calls
and a torch.autograd.Function.

PyTorch supplies device memory and the HIP stream; every step of the solve
runs in the library's HIP kernels.  Functions here only check shapes and
dtypes and pass pointers.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np
import torch

from . import _lib

PRECISIONS = {"fp64": _lib.TG_FP64, "fp32": _lib.TG_FP32_MIXED}


@dataclasses.dataclass
class Stats:
    solves: int
    pcg_its_total: int
    pcg_its_max: int
    status_bits: int
    worst_rel_residual: float


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


class Plan:
    """One grid size, horizon, basis and precision; ``batch`` independent
    problems solved together.

    centres: array [n_p, 3] (shared by the batch) or [batch, n_p, 3].
    precision: "fp64" or "fp32" (FP32 fields and transforms with FP64
    reductions).
    """

    def __init__(self, n: int, nt: int, centres, sigma: float, T: float = 1.0,
                 rtol: float = 1e-8, maxit: int = 1000, ckpt_stride: int = 0,
                 precision: str = "fp64", batch: int = 1, max_hvp_dirs: int = 0,
                 device: str | torch.device = "cuda:0", schedule=None, passes=None):
        L = _lib.lib()
        cen = np.asarray(centres, dtype=np.float64)
        if cen.ndim == 2:
            cen = np.broadcast_to(cen, (batch,) + cen.shape)
        cen = np.ascontiguousarray(cen)
        if cen.shape[0] != batch or cen.shape[2] != 3:
            raise ValueError(f"centres shape {cen.shape} does not match batch {batch}")
        self.n, self.nt, self.T = int(n), int(nt), float(T)
        self.n_p = int(cen.shape[1])
        self.batch = int(batch)
        self.max_hvp_dirs = int(max_hvp_dirs)
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device(device)
        self._cen = cen
        d = _lib.TgDesc(self.n, self.nt, self.T, self.n_p,
                        cen.ctypes.data_as(C.POINTER(C.c_double)), float(sigma),
                        float(rtol), int(maxit), int(ckpt_stride), PRECISIONS[precision],
                        self.batch, self.max_hvp_dirs)
        h = C.c_void_p()
        _lib.check(L.tg_plan_create(C.byref(d), C.byref(h)), "tg_plan_create")
        self._h = h
        nbytes = C.c_size_t()
        _lib.check(L.tg_plan_workspace_bytes(h, C.byref(nbytes)), "tg_plan_workspace_bytes")
        self.workspace_bytes = int(nbytes.value)
        self._ws = None
        self._schedule = schedule
        self._passes_req = dict(passes or {})
        self._passes = {}
        self._keep = ()
        self.generation = 0

    # ------------------------------------------------------------ plumbing
    def _bind(self):
        if self._ws is not None:
            return
        with torch.cuda.device(self.device):
            ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            off = (-ws.data_ptr()) % 256
            self._ws = ws
            _lib.check(_lib.lib().tg_plan_bind(self._h, C.c_void_p(ws.data_ptr() + off),
                                                self.workspace_bytes), "tg_plan_bind")
            passes = self._passes_req
            if self._schedule is not None:
                self.set_schedule(*self._schedule)
            else:
                from . import autotune
                ent = autotune.lookup(autotune.gpu_arch(self.device), self.n, self.precision,
                                      self.batch)
                if ent is not None:
                    self.set_schedule(*ent[0])
                    passes = {**ent[1], **passes}
            for k, (c, o) in passes.items():
                self.set_pass(k, c, o)

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _field(self, x, name):
        if not isinstance(x, torch.Tensor):
            x = torch.as_tensor(np.asarray(x), device=self.device)
        x = x.to(device=self.device, dtype=self.dtype).contiguous()
        if x.numel() != self.batch * self.n ** 3:
            raise ValueError(f"{name}: expected {self.batch} x {self.n}^3 values, got {x.numel()}")
        return x

    def _vec(self, x, count, name):
        if not isinstance(x, torch.Tensor):
            x = torch.as_tensor(np.asarray(x, dtype=np.float64), device=self.device)
        x = x.to(device=self.device, dtype=torch.float64).contiguous()
        if x.numel() != count:
            raise ValueError(f"{name}: expected {count} values, got {x.numel()}")
        return x

    def _shape(self, t):
        return t.view(self.n, self.n, self.n) if self.batch == 1 else \
            t.view(self.batch, self.n, self.n, self.n)

    # ---------------------------------------------------------------- calls
    def forward(self, p, rho_f, k_f, m, m_react=None, phi_mask=None) -> torch.Tensor:
        """c(T) for coefficients p, growth rates rho_f and k_f, diffusion
        field m (the WM map, or sum_i k_i m_i over tissues).  m_react: the
        reaction field sum_i rho_i m_i (default m); phi_mask: multiplies
        Phi p, e.g. 1 - m_CSF (default none)."""
        self._bind()
        p = self._vec(p, self.batch * self.n_p, "p")
        rho = self._vec(rho_f, self.batch, "rho_f")
        kf = self._vec(k_f, self.batch, "k_f")
        m = self._field(m, "m")
        mr = None if m_react is None else self._field(m_react, "m_react")
        mask = None if phi_mask is None else self._field(phi_mask, "phi_mask")
        cT = torch.empty_like(m)
        if mr is None and mask is None:
            st = _lib.lib().tg_forward(self._h, _ptr(p), _ptr(rho), _ptr(kf), _ptr(m),
                                       _ptr(cT), self._stream())
        else:
            st = _lib.lib().tg_forward_fields(self._h, _ptr(p), _ptr(rho), _ptr(kf), _ptr(m),
                                              _ptr(mr) if mr is not None else None,
                                              _ptr(mask) if mask is not None else None,
                                              _ptr(cT), self._stream())
        self._keep = (p, rho, kf, m, mr, mask, cT)
        self.generation += 1
        _lib.check(st, "tg_forward")
        return self._shape(cT)

    def vjp(self, lamT, coupling: bool = False, combine: bool = False):
        """(g_p, g_rho, g_kf) = d<lamT, c(T)>/d(p, rho_f, k_f) of the last
        forward.  coupling=True adds (q_diff, q_react): the derivatives at
        every grid point in the diffusion and reaction fields; with
        combine=True the library returns their sum q_diff + q_react as one
        field instead (the derivative in m when m drives both)."""
        self._bind()
        lam = self._field(lamT, "lamT")
        gp = torch.empty(self.batch * self.n_p, dtype=torch.float64, device=self.device)
        gr = torch.empty(self.batch, dtype=torch.float64, device=self.device)
        gk = torch.empty(self.batch, dtype=torch.float64, device=self.device)
        if not coupling:
            _lib.check(_lib.lib().tg_vjp(self._h, _ptr(lam), _ptr(gp), _ptr(gr), _ptr(gk),
                                         self._stream()), "tg_vjp")
            return self._vecs(gp, gr, gk)
        qd = torch.empty_like(lam)
        qr = None if combine else torch.empty_like(lam)
        _lib.check(_lib.lib().tg_vjp_coupling(self._h, _ptr(lam), _ptr(gp), _ptr(gr), _ptr(gk),
                                              _ptr(qd), _ptr(qr), 1 if combine else 0,
                                              self._stream()),
                   "tg_vjp_coupling")
        if combine:
            return (*self._vecs(gp, gr, gk), self._shape(qd))
        return (*self._vecs(gp, gr, gk), self._shape(qd), self._shape(qr))

    def adjoint_misfit(self, c_obs, labels=None):
        """(J, g_p, g_rho, g_kf) of J = 1/2 h^3 sum (c(T) - c_obs)^2; with
        labels = (m_lab, m_pat), each [batch][L][n^3] (or [L][n^3] for one
        problem), J adds 1/2 h^3 sum_l sum (m_l (1 - c(T)) - mP_l)^2."""
        self._bind()
        d = self._field(c_obs, "c_obs")
        J = torch.empty(self.batch, dtype=torch.float64, device=self.device)
        gp = torch.empty(self.batch * self.n_p, dtype=torch.float64, device=self.device)
        gr = torch.empty(self.batch, dtype=torch.float64, device=self.device)
        gk = torch.empty(self.batch, dtype=torch.float64, device=self.device)
        if labels is None:
            st = _lib.lib().tg_adjoint_misfit(self._h, _ptr(d), _ptr(J), _ptr(gp), _ptr(gr),
                                              _ptr(gk), self._stream())
        else:
            ml, mp = (self._labels(x, name) for x, name in zip(labels, ("m_lab", "m_pat")))
            if ml.shape != mp.shape:
                raise ValueError("m_lab and m_pat must have the same shape")
            st = _lib.lib().tg_adjoint_misfit_labels(
                self._h, _ptr(d), ml.shape[1], _ptr(ml), _ptr(mp), _ptr(J), _ptr(gp),
                _ptr(gr), _ptr(gk), self._stream())
        _lib.check(st, "tg_adjoint_misfit")
        gp, gr, gk = self._vecs(gp, gr, gk)
        return (J[0] if self.batch == 1 else J), gp, gr, gk

    def _labels(self, x, name):
        if not isinstance(x, torch.Tensor):
            x = torch.as_tensor(np.asarray(x), device=self.device)
        x = x.to(device=self.device, dtype=self.dtype).contiguous()
        n3 = self.n ** 3
        if x.numel() % (self.batch * n3) != 0 or x.numel() == 0:
            raise ValueError(f"{name}: expected [{self.batch}][L][{self.n}^3] values")
        return x.view(self.batch, x.numel() // (self.batch * n3), n3)

    # -------------------------------------------------- registration transport
    def transport(self, v, m0, nt_r: int, w=None) -> torch.Tensor:
        """Semi-Lagrangian transport of the label fields m0 ([L][n^3] or
        [L, n, n, n]) by the stationary velocity v ([3][n^3]) over nt_r
        steps; returns m(1) as [L, n, n, n].  w = div v (default 0) is
        used by transport_adjoint.  Needs a single-problem plan."""
        self._bind()
        n3 = self.n ** 3
        v = self._many(v, 3, "v")
        m0 = self._many(m0, None, "m0")
        L = m0.numel() // n3
        wt = None if w is None else self._many(w, 1, "w")
        nb = C.c_size_t()
        _lib.check(_lib.lib().tg_transport_workspace_bytes(self._h, int(nt_r), L, C.byref(nb)),
                   "tg_transport_workspace_bytes")
        tws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        off = (-tws.data_ptr()) % 256
        m1 = torch.empty_like(m0)
        _lib.check(_lib.lib().tg_transport(self._h, int(nt_r), L, _ptr(v), _ptr(wt), _ptr(m0),
                                           _ptr(m1), C.c_void_p(tws.data_ptr() + off), nb.value,
                                           self._stream()), "tg_transport")
        self._tkeep = (v, wt, m0, tws)
        return m1.view(L, self.n, self.n, self.n)

    def transport_adjoint(self, lam1):
        """Adjoint of the last transport from lam(1) ([L][n^3]): returns
        (lam(0) as [L, n, n, n], body force as [3, n, n, n])."""
        self._bind()
        lam1 = self._many(lam1, None, "lam1")
        L = lam1.numel() // self.n ** 3
        lam0 = torch.empty_like(lam1)
        body = torch.empty(3 * self.n ** 3, dtype=self.dtype, device=self.device)
        _lib.check(_lib.lib().tg_transport_adjoint(self._h, _ptr(lam1), _ptr(lam0), _ptr(body),
                                                   self._stream()), "tg_transport_adjoint")
        n = self.n
        return lam0.view(L, n, n, n), body.view(3, n, n, n)

    def _many(self, x, count, name):
        if not isinstance(x, torch.Tensor):
            x = torch.as_tensor(np.asarray(x), device=self.device)
        x = x.to(device=self.device, dtype=self.dtype).contiguous()
        n3 = self.n ** 3
        if x.numel() == 0 or x.numel() % n3 or (count is not None and x.numel() != count * n3):
            raise ValueError(f"{name}: expected {count or 'L'} fields of {self.n}^3 values")
        return x

    def hessvec(self, V) -> torch.Tensor:
        """Gauss-Newton Hessian products H V[d] for V of shape [ndir, n_p]."""
        self._bind()
        V = torch.as_tensor(V, dtype=torch.float64, device=self.device).contiguous()
        if V.ndim == 1:
            V = V[None]
        ndir = V.shape[0]
        if V.shape[1] != self.n_p:
            raise ValueError(f"V: expected [ndir, {self.n_p}], got {tuple(V.shape)}")
        HV = torch.empty_like(V)
        _lib.check(_lib.lib().tg_hessvec_gn(self._h, ndir, _ptr(V), _ptr(HV), self._stream()),
                   "tg_hessvec_gn")
        return HV

    def stats(self) -> Stats:
        s = _lib.TgSolveStats()
        _lib.check(_lib.lib().tg_stats(self._h, C.byref(s)), "tg_stats")
        return Stats(s.solves, s.pcg_its_total, s.pcg_its_max, s.status_bits,
                     s.worst_rel_residual)

    def set_schedule(self, pencils: int = 0, z_waves: int = 0, slabs: int = 0,
                     waves_per_simd: int = 0):
        """Choose the transform launch schedule (0 = default)."""
        if self._ws is None:
            self._schedule = (int(pencils), int(z_waves), int(slabs), int(waves_per_simd))
            self._bind()
            return
        _lib.check(_lib.lib().tg_plan_set_schedule(self._h, int(pencils), int(z_waves),
                                                    int(slabs), int(waves_per_simd)),
                   "tg_plan_set_schedule")
        self._passes = {}

    def get_schedule(self):
        self._bind()
        v = [C.c_int() for _ in range(4)]
        _lib.check(_lib.lib().tg_plan_get_schedule(self._h, *[C.byref(x) for x in v]),
                   "tg_plan_get_schedule")
        return tuple(x.value for x in v)

    KERNELS = {"x_inv_grad": 1, "y_inv_grad": 2, "z_matvec": 3, "y_fwd_div": 4,
               "x_fwd_div": 5}

    def set_pass(self, kernel: str, pencils: int, waves_per_simd: int):
        """Tile shape of one PCG pass (after set_schedule); pencils 0 for z_matvec."""
        self._bind()
        _lib.check(_lib.lib().tg_plan_set_pass(self._h, self.KERNELS[kernel], int(pencils),
                                                int(waves_per_simd)), "tg_plan_set_pass")
        self._passes[kernel] = (int(pencils), int(waves_per_simd))

    def get_pass(self, kernel: str):
        self._bind()
        c, o = C.c_int(), C.c_int()
        _lib.check(_lib.lib().tg_plan_get_pass(self._h, self.KERNELS[kernel], C.byref(c),
                                                C.byref(o)), "tg_plan_get_pass")
        return c.value, o.value

    def kernel_timer(self, name: str | None, every: int = 1):
        """Bracket the launches of one PCG-iteration kernel with HIP events,
        in one Crank-Nicolson solve in `every` (1: all of them)."""
        self._bind()
        kid = 0 if name is None else self.KERNELS[name]
        _lib.check(_lib.lib().tg_kernel_timer(self._h, kid, int(every)), "tg_kernel_timer")

    def kernel_timer_read(self):
        """(total ms, launches, algorithmic bytes moved by the timed launches)."""
        ms, n, b = C.c_double(), C.c_longlong(), C.c_double()
        _lib.check(_lib.lib().tg_kernel_timer_read(self._h, C.byref(ms), C.byref(n), C.byref(b)),
                   "tg_kernel_timer_read")
        return ms.value, n.value, b.value

    def _vecs(self, gp, gr, gk):
        if self.batch == 1:
            return gp, gr[0], gk[0]
        return gp.view(self.batch, self.n_p), gr, gk

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                if self._ws is not None:
                    torch.cuda.synchronize(self.device)
                _lib.lib().tg_plan_destroy(h)
            except Exception:
                pass
            self._h = None


class TumorSolve(torch.autograd.Function):
    """c(T) = TumorSolve.apply(p, rho_f, k_f, m, plan); differentiable in
    p, rho_f, k_f and the white-matter map m through the library's discrete
    adjoint (m's gradient is the coupling field, q_diff + q_react)."""

    @staticmethod
    def forward(ctx, p, rho_f, k_f, m, plan: Plan):
        cT = plan.forward(p.detach(), rho_f.detach(), k_f.detach(), m.detach())
        ctx.plan = plan
        ctx.gen = plan.generation
        ctx.save_for_backward(p.detach(), rho_f.detach(), k_f.detach(), m.detach())
        return cT.clone()

    @staticmethod
    def backward(ctx, grad_cT):
        plan: Plan = ctx.plan
        if plan.generation != ctx.gen:
            # another forward used the plan since: rebuild this trajectory
            p, rho, kf, m = ctx.saved_tensors
            plan.forward(p, rho, kf, m)
            ctx.gen = plan.generation
        p, rho, kf, m = ctx.saved_tensors
        gm = None
        if ctx.needs_input_grad[3]:
            # m drives both coefficients: the library returns dJ/dm = q_diff + q_react
            gp, gr, gk, q = plan.vjp(grad_cT.detach(), coupling=True, combine=True)
            gm = q.reshape(m.shape).to(m.dtype)
        else:
            gp, gr, gk = plan.vjp(grad_cT.detach())
        return (gp.view_as(p).to(p.dtype), gr.reshape(rho.shape).to(rho.dtype),
                gk.reshape(kf.shape).to(kf.dtype), gm, None)


class TumorSolveFields(torch.autograd.Function):
    """c(T) = TumorSolveFields.apply(p, rho_f, k_f, m_diff, m_react,
    phi_mask, plan): the full coefficient model (tissue-weighted diffusion
    field m_diff and reaction field m_react, basis masked by phi_mask,
    which may be None).  Differentiable in p, rho_f, k_f, m_diff and
    m_react through the library's discrete adjoint (the field gradients are
    the coupling fields q_diff and q_react); phi_mask is data."""

    @staticmethod
    def forward(ctx, p, rho_f, k_f, m_diff, m_react, phi_mask, plan: Plan):
        mask = None if phi_mask is None else phi_mask.detach()
        args = (p.detach(), rho_f.detach(), k_f.detach(), m_diff.detach(), m_react.detach())
        cT = plan.forward(*args[:4], m_react=args[4], phi_mask=mask)
        ctx.plan = plan
        ctx.gen = plan.generation
        ctx.mask = mask
        ctx.save_for_backward(*args)
        return cT.clone()

    @staticmethod
    def backward(ctx, grad_cT):
        plan: Plan = ctx.plan
        p, rho, kf, md, mr = ctx.saved_tensors
        if plan.generation != ctx.gen:
            # another forward used the plan since: rebuild this trajectory
            plan.forward(p, rho, kf, md, m_react=mr, phi_mask=ctx.mask)
            ctx.gen = plan.generation
        gd = gr_field = None
        if ctx.needs_input_grad[3] or ctx.needs_input_grad[4]:
            gp, gr, gk, qd, qr = plan.vjp(grad_cT.detach(), coupling=True)
            gd = qd.reshape(md.shape).to(md.dtype) if ctx.needs_input_grad[3] else None
            gr_field = qr.reshape(mr.shape).to(mr.dtype) if ctx.needs_input_grad[4] else None
        else:
            gp, gr, gk = plan.vjp(grad_cT.detach())
        return (gp.view_as(p).to(p.dtype), gr.reshape(rho.shape).to(rho.dtype),
                gk.reshape(kf.shape).to(kf.dtype), gd, gr_field, None, None)


class BatchGraph:
    """Gradient evaluations (forward + misfit + adjoint) of several plans
    captured into one HIP graph and replayed with one launch.

    items: list of (plan, p, rho_f, k_f, m, c_obs) with per-plan batched
    inputs.  Each plan needs one eager gradient before capture (it sizes the
    fixed PCG iteration budget) unless ``pcg_budget`` is given.  Inputs are
    copied into buffers owned by this object; ``update`` rewrites them in
    place between launches.
    """

    def __init__(self, items, pcg_budget: int = 0):
        self.plans = [it[0] for it in items]
        dev = self.plans[0].device
        self.device = dev
        self.stream = torch.cuda.Stream(device=dev)
        self._bufs = []
        ios = (_lib.TgBatchIo * len(items))()
        for i, (plan, p, rho, kf, m, cobs) in enumerate(items):
            plan._bind()
            b = {
                "p": plan._vec(p, plan.batch * plan.n_p, "p").clone(),
                "rho": plan._vec(rho, plan.batch, "rho_f").clone(),
                "kf": plan._vec(kf, plan.batch, "k_f").clone(),
                "m": plan._field(m, "m").clone(),
                "cobs": plan._field(cobs, "c_obs").clone(),
            }
            b["cT"] = torch.empty_like(b["m"])
            b["J"] = torch.empty(plan.batch, dtype=torch.float64, device=dev)
            b["gp"] = torch.empty(plan.batch * plan.n_p, dtype=torch.float64, device=dev)
            b["grho"] = torch.empty(plan.batch, dtype=torch.float64, device=dev)
            b["gkf"] = torch.empty(plan.batch, dtype=torch.float64, device=dev)
            for f, k in (("d_p", "p"), ("d_rho_f", "rho"), ("d_k_f", "kf"), ("d_m", "m"),
                         ("d_cT", "cT"), ("d_cobs", "cobs"), ("d_J", "J"), ("d_gp", "gp"),
                         ("d_grho", "grho"), ("d_gkf", "gkf")):
                setattr(ios[i], f, b[k].data_ptr())
            self._bufs.append(b)
        handles = (C.c_void_p * len(items))(*[pl._h.value for pl in self.plans])
        h = C.c_void_p()
        torch.cuda.synchronize(dev)
        _lib.check(_lib.lib().tg_batch_capture(len(items), handles, ios, int(pcg_budget),
                                               C.c_void_p(self.stream.cuda_stream), C.byref(h)),
                   "tg_batch_capture")
        self._h = h
        for pl, b in zip(self.plans, self._bufs):
            pl._keep = (b["p"], b["rho"], b["kf"], b["m"], b["cT"])
            pl.generation += 1

    def update(self, i, p=None, rho_f=None, k_f=None, m=None, c_obs=None):
        b, pl = self._bufs[i], self.plans[i]
        if p is not None:
            b["p"].copy_(pl._vec(p, pl.batch * pl.n_p, "p"))
        if rho_f is not None:
            b["rho"].copy_(pl._vec(rho_f, pl.batch, "rho_f"))
        if k_f is not None:
            b["kf"].copy_(pl._vec(k_f, pl.batch, "k_f"))
        if m is not None:
            b["m"].copy_(pl._field(m, "m"))
        if c_obs is not None:
            b["cobs"].copy_(pl._field(c_obs, "c_obs"))

    def launch(self):
        """Replay the graph on this object's stream, ordered after the
        current stream's prior work; the current stream waits for it."""
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        _lib.check(_lib.lib().tg_batch_launch(self._h, C.c_void_p(self.stream.cuda_stream)),
                   "tg_batch_launch")
        cur.wait_stream(self.stream)

    def results(self, check: bool = True):
        """[(J, g_p, g_rho, g_kf)] per plan (device tensors, batched).

        check (default): read each plan's solve statistics after the replay
        and raise if a solve hit its captured iteration budget or pcg_maxit
        (TG_ERR_NOT_CONVERGED), broke down or went non-finite
        (TG_ERR_NUMERIC), or met an invalid k_f / rho_f (TG_ERR_ARG): a
        replay whose inputs need more iterations than the budget otherwise
        returns unconverged gradients.  Synchronizes the plans' stream."""
        if check:
            for i, pl in enumerate(self.plans):
                bits = pl.stats().status_bits
                if bits:
                    st = (_lib.TG_ERR_ARG if bits & 8 else
                          _lib.TG_ERR_NUMERIC if bits & 6 else _lib.TG_ERR_NOT_CONVERGED)
                    _lib.check(st, f"BatchGraph plan {i} (status bits {bits})")
        out = []
        for pl, b in zip(self.plans, self._bufs):
            out.append((b["J"], b["gp"].view(pl.batch, pl.n_p), b["grho"], b["gkf"]))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
                _lib.lib().tg_batch_destroy(h)
            except Exception:
                pass
            self._h = None
