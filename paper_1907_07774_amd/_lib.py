"""ctypes declarations of the libtumorgrad C-ABI (include/tumorgrad.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtumorgrad.so")

TG_OK = 0
TG_ERR_ARG = 1
TG_ERR_STATE = 2
TG_ERR_NOT_CONVERGED = 3
TG_ERR_NUMERIC = 4
TG_ERR_HIP = 5
TG_ERR_WORKSPACE = 6
TG_ERR_SCRATCH_LIMIT = 7

TG_FP64 = 0
TG_FP32_MIXED = 1

EXPORTS = (
    "tg_plan_create", "tg_plan_workspace_bytes", "tg_plan_bind", "tg_forward",
    "tg_vjp", "tg_adjoint_misfit", "tg_hessvec_gn", "tg_stats",
    "tg_status_string", "tg_plan_destroy", "tg_version", "tg_kernel_timer",
    "tg_kernel_timer_read", "tg_plan_set_schedule", "tg_plan_get_schedule",
    "tg_plan_set_pass", "tg_plan_get_pass", "tg_forward_fields", "tg_adjoint_misfit_labels",
    "tg_vjp_coupling", "tg_transport_workspace_bytes", "tg_transport", "tg_transport_adjoint",
    "tg_stream_probe", "tg_forward_static",
    "tg_batch_capture", "tg_batch_launch", "tg_batch_destroy",
)


class TgDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("nt", C.c_int), ("T", C.c_double), ("n_p", C.c_int),
        ("centres", C.POINTER(C.c_double)), ("sigma", C.c_double),
        ("pcg_rtol", C.c_double), ("pcg_maxit", C.c_int), ("ckpt_stride", C.c_int),
        ("prec", C.c_int), ("batch", C.c_int), ("max_hvp_dirs", C.c_int),
    ]


class TgBatchIo(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in (
        "d_p", "d_rho_f", "d_k_f", "d_m", "d_cT", "d_cobs", "d_J", "d_gp", "d_grho", "d_gkf")]


class TgSolveStats(C.Structure):
    _fields_ = [
        ("solves", C.c_int), ("pcg_its_total", C.c_int), ("pcg_its_max", C.c_int),
        ("status_bits", C.c_int), ("worst_rel_residual", C.c_double),
    ]


class TumorGradError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load libtumorgrad.so once.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    vp, dp, sz = C.c_void_p, C.POINTER(C.c_double), C.c_size_t
    L.tg_plan_create.argtypes = [C.POINTER(TgDesc), C.POINTER(vp)]
    L.tg_plan_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
    L.tg_plan_bind.argtypes = [vp, vp, sz]
    L.tg_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.tg_forward_static.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.tg_vjp.argtypes = [vp, vp, vp, vp, vp, vp]
    L.tg_adjoint_misfit.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.tg_forward_fields.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.tg_vjp_coupling.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_int, vp]
    L.tg_transport_workspace_bytes.argtypes = [vp, C.c_int, C.c_int, C.POINTER(sz)]
    L.tg_transport.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, vp, vp, sz, vp]
    L.tg_transport_adjoint.argtypes = [vp, vp, vp, vp, vp]
    L.tg_stream_probe.argtypes = [vp, sz, sz, C.c_int, dp, vp]
    L.tg_adjoint_misfit_labels.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, vp, vp, vp]
    L.tg_hessvec_gn.argtypes = [vp, C.c_int, vp, vp, vp]
    L.tg_stats.argtypes = [vp, C.POINTER(TgSolveStats)]
    L.tg_status_string.argtypes = [C.c_int]
    L.tg_status_string.restype = C.c_char_p
    L.tg_plan_destroy.argtypes = [vp]
    L.tg_plan_destroy.restype = None
    L.tg_version.restype = C.c_int
    L.tg_kernel_timer.argtypes = [vp, C.c_int, C.c_int]
    L.tg_kernel_timer_read.argtypes = [vp, dp, C.POINTER(C.c_longlong), dp]
    L.tg_batch_capture.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(TgBatchIo), C.c_int, vp,
                                   C.POINTER(vp)]
    L.tg_batch_launch.argtypes = [vp, vp]
    L.tg_batch_destroy.argtypes = [vp]
    L.tg_batch_destroy.restype = None
    L.tg_plan_set_schedule.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
    L.tg_plan_get_schedule.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.tg_plan_set_pass.argtypes = [vp, C.c_int, C.c_int, C.c_int]
    L.tg_plan_get_pass.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    for name in ("tg_plan_create", "tg_plan_workspace_bytes", "tg_plan_bind", "tg_forward",
                 "tg_forward_static",
                 "tg_vjp", "tg_adjoint_misfit", "tg_hessvec_gn", "tg_stats",
                 "tg_kernel_timer", "tg_kernel_timer_read", "tg_plan_set_schedule",
                 "tg_plan_get_schedule", "tg_plan_set_pass", "tg_plan_get_pass",
                 "tg_batch_capture", "tg_batch_launch"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(status: int, where: str, allow=()) -> int:
    if status == TG_OK or status in allow:
        return status
    msg = lib().tg_status_string(status).decode()
    raise TumorGradError(status, where, msg)
