"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/tumorgrad.h, and rejects bad arguments on the
host before launching anything."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1907_07774_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "tumorgrad.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tg_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = _lib.lib()
    names = header_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L, n), n
    assert set(_lib.EXPORTS) == set(names)


def test_version_and_status_strings():
    L = _lib.lib()
    assert L.tg_version() == 1
    for s in range(8):
        assert len(L.tg_status_string(s)) > 0


def make_desc(**kw):
    cen = np.zeros((kw.pop("batch", 1), kw.pop("n_p", 8), 3))
    d = dict(n=16, nt=4, T=1.0, sigma=0.2, pcg_rtol=1e-8, pcg_maxit=100, ckpt_stride=0,
             prec=_lib.TG_FP64, batch=cen.shape[0], max_hvp_dirs=0)
    d.update(kw)
    desc = _lib.TgDesc(d["n"], d["nt"], d["T"], cen.shape[1],
                       cen.ctypes.data_as(C.POINTER(C.c_double)), d["sigma"], d["pcg_rtol"],
                       d["pcg_maxit"], d["ckpt_stride"], d["prec"], d["batch"], d["max_hvp_dirs"])
    return desc, cen


def create(**kw):
    desc, cen = make_desc(**kw)
    h = C.c_void_p()
    st = _lib.lib().tg_plan_create(C.byref(desc), C.byref(h))
    return st, h


@pytest.mark.parametrize("bad", [dict(n=12), dict(n=512), dict(n=4), dict(nt=0), dict(T=0.0),
                                 dict(T=float("nan")), dict(sigma=-1.0), dict(pcg_rtol=0.0),
                                 dict(pcg_rtol=1.5), dict(pcg_maxit=0), dict(ckpt_stride=-1),
                                 dict(prec=7), dict(max_hvp_dirs=-2)])
def test_plan_create_rejects_bad_descriptors(bad):
    st, h = create(**bad)
    assert st == _lib.TG_ERR_ARG
    assert not h.value


def test_plan_create_and_workspace_size():
    L = _lib.lib()
    st, h = create(n=32, nt=8, ckpt_stride=4, max_hvp_dirs=2)
    assert st == _lib.TG_OK
    nb = C.c_size_t()
    assert L.tg_plan_workspace_bytes(h, C.byref(nb)) == _lib.TG_OK
    # 7 spectra, 7 spectra per direction, checkpoints, segment, adjoint; FP64
    field = 32 ** 3 * 8
    assert nb.value >= (7 + 7 * 2 + 2 + 2 + 4 + 4 + 2) * field
    # unbound plan: calls fail on the host without touching a GPU
    assert L.tg_forward(h, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                        C.c_void_p(8), None) == _lib.TG_ERR_WORKSPACE
    assert L.tg_vjp(h, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                    None) == _lib.TG_ERR_STATE
    assert L.tg_hessvec_gn(h, 1, C.c_void_p(8), C.c_void_p(8), None) == _lib.TG_ERR_STATE
    assert L.tg_hessvec_gn(h, 3, C.c_void_p(8), C.c_void_p(8), None) == _lib.TG_ERR_ARG
    assert L.tg_plan_bind(h, None, nb.value) == _lib.TG_ERR_WORKSPACE
    assert L.tg_plan_bind(h, C.c_void_p(4096 + 8), nb.value) == _lib.TG_ERR_WORKSPACE
    assert L.tg_plan_bind(h, C.c_void_p(4096), nb.value - 1) == _lib.TG_ERR_WORKSPACE
    assert L.tg_forward(h, None, None, None, None, None, None) == _lib.TG_ERR_ARG
    L.tg_plan_destroy(h)


def test_schedule_calls_need_a_bound_plan():
    L = _lib.lib()
    st, h = create(n=32, nt=4)
    assert st == _lib.TG_OK
    c, o = C.c_int(), C.c_int()
    assert L.tg_plan_set_schedule(h, 16, 1, 1, 1) == _lib.TG_ERR_WORKSPACE
    assert L.tg_plan_set_pass(h, 1, 16, 1) == _lib.TG_ERR_WORKSPACE
    assert L.tg_plan_get_pass(h, 1, C.byref(c), C.byref(o)) == _lib.TG_ERR_WORKSPACE
    assert L.tg_plan_set_pass(None, 1, 16, 1) == _lib.TG_ERR_ARG
    assert L.tg_plan_get_pass(h, 1, None, C.byref(o)) == _lib.TG_ERR_ARG
    # kernel timer: argument checks before the workspace check
    assert L.tg_kernel_timer(h, 3, 0) == _lib.TG_ERR_ARG
    assert L.tg_kernel_timer(h, 99, 1) == _lib.TG_ERR_ARG
    assert L.tg_kernel_timer(None, 3, 1) == _lib.TG_ERR_ARG
    assert L.tg_kernel_timer(h, 3, 8) == _lib.TG_ERR_WORKSPACE
    L.tg_plan_destroy(h)


def test_fp32_workspace_is_half_of_fp64():
    L = _lib.lib()
    sizes = []
    for prec in (_lib.TG_FP64, _lib.TG_FP32_MIXED):
        st, h = create(n=64, nt=8, prec=prec)
        nb = C.c_size_t()
        L.tg_plan_workspace_bytes(h, C.byref(nb))
        sizes.append(nb.value)
        L.tg_plan_destroy(h)
    assert sizes[1] < 0.6 * sizes[0]


def test_nonfinite_centres_rejected():
    desc, cen = make_desc()
    cen[0, 0, 0] = np.nan
    h = C.c_void_p()
    assert _lib.lib().tg_plan_create(C.byref(desc), C.byref(h)) == _lib.TG_ERR_ARG


def test_model_and_coupling_calls_check_on_the_host():
    """tg_forward_fields, tg_vjp_coupling and tg_adjoint_misfit_labels on an
    unbound plan: argument errors first, then missing workspace or state."""
    L = _lib.lib()
    st, h = create(n=32, nt=4)
    assert st == _lib.TG_OK
    p = C.c_void_p(8)
    assert L.tg_forward_fields(h, p, p, p, None, p, p, p, None) == _lib.TG_ERR_ARG
    assert L.tg_forward_fields(h, p, p, p, p, None, None, None, None) == _lib.TG_ERR_ARG
    assert L.tg_forward_fields(h, p, p, p, p, None, None, p, None) == _lib.TG_ERR_WORKSPACE
    assert L.tg_forward_fields(h, p, p, p, p, p, p, p, None) == _lib.TG_ERR_WORKSPACE
    assert L.tg_vjp_coupling(h, p, p, p, p, p, p, 0, None) == _lib.TG_ERR_STATE
    assert L.tg_vjp_coupling(h, p, p, p, p, p, None, 1, None) == _lib.TG_ERR_STATE
    assert L.tg_vjp_coupling(h, None, p, p, p, p, p, 0, None) == _lib.TG_ERR_ARG
    assert L.tg_vjp_coupling(h, p, p, p, None, p, p, 0, None) == _lib.TG_ERR_ARG
    # combine = 1 takes one output field: d_q_diff set, d_q_react NULL
    assert L.tg_vjp_coupling(h, p, p, p, p, p, p, 1, None) == _lib.TG_ERR_ARG
    assert L.tg_vjp_coupling(h, p, p, p, p, None, None, 1, None) == _lib.TG_ERR_ARG
    assert L.tg_vjp_coupling(h, p, p, p, p, p, p, 2, None) == _lib.TG_ERR_ARG
    assert L.tg_adjoint_misfit_labels(h, p, 0, None, None, p, p, p, p, None) == _lib.TG_ERR_STATE
    assert L.tg_adjoint_misfit_labels(h, p, 3, p, p, p, p, p, p, None) == _lib.TG_ERR_STATE
    assert L.tg_adjoint_misfit_labels(h, p, -1, p, p, p, p, p, p, None) == _lib.TG_ERR_ARG
    assert L.tg_adjoint_misfit_labels(h, p, 2, None, p, p, p, p, p, None) == _lib.TG_ERR_ARG
    assert L.tg_adjoint_misfit_labels(h, p, 2, p, None, p, p, p, p, None) == _lib.TG_ERR_ARG
    assert L.tg_adjoint_misfit_labels(h, None, 0, None, None, p, p, p, p,
                                      None) == _lib.TG_ERR_ARG
    L.tg_plan_destroy(h)


@pytest.mark.parametrize("prec,es", [(_lib.TG_FP64, 8), (_lib.TG_FP32_MIXED, 4)])
def test_transport_workspace_size_and_host_errors(prec, es):
    """Transport workspace: every time level of every label, the velocity's
    feet and scratch (9 fields) and two more fields per label."""
    L = _lib.lib()
    st, h = create(n=32, nt=4, prec=prec)
    assert st == _lib.TG_OK
    nb = C.c_size_t()
    for nt_r, nl in ((1, 1), (4, 3), (8, 2)):
        assert L.tg_transport_workspace_bytes(h, nt_r, nl, C.byref(nb)) == _lib.TG_OK
        assert nb.value == ((nt_r + 1) * nl + 9 + 2 * nl) * 32 ** 3 * es
    assert L.tg_transport_workspace_bytes(h, 0, 1, C.byref(nb)) == _lib.TG_ERR_ARG
    assert L.tg_transport_workspace_bytes(h, 1, 0, C.byref(nb)) == _lib.TG_ERR_ARG
    assert L.tg_transport_workspace_bytes(h, 1, 1, None) == _lib.TG_ERR_ARG
    L.tg_transport_workspace_bytes(h, 4, 2, C.byref(nb))
    need = nb.value
    p, ws = C.c_void_p(8), C.c_void_p(1 << 20)
    assert L.tg_transport(h, 4, 2, p, None, p, p, ws, need, None) == _lib.TG_ERR_WORKSPACE
    assert L.tg_transport(h, 4, 2, p, None, p, p, ws, need - 1, None) == _lib.TG_ERR_WORKSPACE
    assert L.tg_transport(h, 4, 2, p, None, p, p, C.c_void_p((1 << 20) + 64), need,
                          None) == _lib.TG_ERR_WORKSPACE
    assert L.tg_transport(h, 0, 2, p, None, p, p, ws, need, None) == _lib.TG_ERR_ARG
    assert L.tg_transport(h, 4, 0, p, None, p, p, ws, need, None) == _lib.TG_ERR_ARG
    assert L.tg_transport(h, 4, 2, None, None, p, p, ws, need, None) == _lib.TG_ERR_ARG
    assert L.tg_transport(h, 4, 2, p, None, None, p, ws, need, None) == _lib.TG_ERR_ARG
    assert L.tg_transport(h, 4, 2, p, None, p, p, None, need, None) == _lib.TG_ERR_ARG
    assert L.tg_transport_adjoint(h, p, p, p, None) == _lib.TG_ERR_STATE
    assert L.tg_transport_adjoint(h, p, None, p, None) == _lib.TG_ERR_ARG
    assert L.tg_transport_adjoint(h, p, p, None, None) == _lib.TG_ERR_ARG
    L.tg_plan_destroy(h)
    st, hb = create(n=32, nt=4, prec=prec, batch=2)
    assert st == _lib.TG_OK
    assert L.tg_transport(hb, 4, 2, p, None, p, p, ws, need, None) == _lib.TG_ERR_ARG
    L.tg_plan_destroy(hb)


def test_stream_probe_rejects_bad_arguments():
    L = _lib.lib()
    out = C.c_double()
    buf = C.c_void_p(1 << 20)
    f = 1 << 16
    assert L.tg_stream_probe(None, 7 * f, f, 1, C.byref(out), None) == _lib.TG_ERR_ARG
    assert L.tg_stream_probe(buf, 7 * f, f, 1, None, None) == _lib.TG_ERR_ARG
    assert L.tg_stream_probe(buf, 7 * f, f, 0, C.byref(out), None) == _lib.TG_ERR_ARG
    assert L.tg_stream_probe(buf, 7 * f - 16, f, 1, C.byref(out), None) == _lib.TG_ERR_ARG
    assert L.tg_stream_probe(buf, 7 * 512, 512, 1, C.byref(out), None) == _lib.TG_ERR_ARG
    assert L.tg_stream_probe(buf, 7 * (f + 8), f + 8, 1, C.byref(out), None) == _lib.TG_ERR_ARG
    assert L.tg_stream_probe(C.c_void_p((1 << 20) + 8), 7 * f, f, 1, C.byref(out),
                             None) == _lib.TG_ERR_ARG


def test_forward_static_host_errors():
    """tg_forward_static rejects null arguments and plans whose workspace
    exceeds the static scratch on the host, before it looks up the scratch
    or launches anything."""
    L = _lib.lib()
    one = C.c_void_p(8)
    st, h = create(n=16, nt=4)
    assert st == _lib.TG_OK
    assert L.tg_forward_static(h, None, one, one, one, one, None) == _lib.TG_ERR_ARG
    assert L.tg_forward_static(h, one, one, one, one, None, None) == _lib.TG_ERR_ARG
    assert L.tg_forward_static(None, one, one, one, one, one, None) == _lib.TG_ERR_ARG
    L.tg_plan_destroy(h)
    # 64^3 FP64 keeping every state: about 91 MiB of workspace
    st, big = create(n=64, nt=16, ckpt_stride=0)
    assert st == _lib.TG_OK
    nb = C.c_size_t()
    assert L.tg_plan_workspace_bytes(big, C.byref(nb)) == _lib.TG_OK
    assert nb.value > 64 << 20
    assert L.tg_forward_static(big, one, one, one, one, one, None) == _lib.TG_ERR_SCRATCH_LIMIT
    assert b"static scratch" in L.tg_status_string(_lib.TG_ERR_SCRATCH_LIMIT)
    L.tg_plan_destroy(big)
