"""ctypes declarations of the C ABI in include/grav.h (one-to-one)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgrav.so")

GRAV_OK, GRAV_EINVAL, GRAV_ENOMEM, GRAV_EDEVICE, GRAV_ENOCONV, GRAV_EBUSY, GRAV_ECANCELED = range(7)
GRAV_FP64, GRAV_MIXED, GRAV_MIXED_BF16X3, GRAV_FP32_VALU = range(4)
OP_FORWARD, OP_ADJOINT, OP_DATASPACE, OP_TRACE, OP_INVERT, OP_FORWARD_MULTI, OP_TREND, OP_SECTIONS = range(8)
GRAV_TREND_SECTION, GRAV_TREND_DOMAIN = range(2)
GRAV_GAMMA = 6.674e-11
GRAV_STATIC_SCRATCH_BYTES = 128 << 20

_c_dp = ctypes.POINTER(ctypes.c_double)


class CMesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("xn", ctypes.c_void_p), ("yn", ctypes.c_void_p), ("zn", ctypes.c_void_p)]


class CObs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p)]


class CtxOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_uint64)]


class CgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("fixed_iters", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("max_cycles", ctypes.c_int32),
                ("max_halvings", ctypes.c_int32), ("history_cap", ctypes.c_int32),
                ("history", ctypes.POINTER(ctypes.c_double)), ("y0", ctypes.c_void_p),
                ("y_out", ctypes.c_void_p), ("graph", ctypes.c_int32)]


class CgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("relres", ctypes.c_double),
                ("lambda_used", ctypes.c_double), ("trace", ctypes.c_double),
                ("cycles", ctypes.c_int32), ("halvings", ctypes.c_int32)]


class SectionOpts(ctypes.Structure):
    _fields_ = [("nsec", ctypes.c_int32), ("ysplit", ctypes.POINTER(ctypes.c_int32)),
                ("data_degree", ctypes.c_int32), ("data_scope", ctypes.c_int32),
                ("model_degree", ctypes.c_int32)]


class GravRequest(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("mesh", CMesh), ("obs", CObs), ("m", ctypes.c_void_p),
                ("d", ctypes.c_void_p), ("d_obs", ctypes.c_void_p), ("wdepth", ctypes.c_void_p),
                ("lam", ctypes.c_double), ("cg", CgOpts), ("m_out", ctypes.c_void_p),
                ("stream", ctypes.c_void_p)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("relres", ctypes.c_double),
                ("lambda_used", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double), ("state_bytes", ctypes.c_uint64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("budget_bytes", ctypes.c_uint64)]


class GravError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"grav error {code}: {msg}")
        self.code = code


def _load():
    # torch ships its own HIP runtime (SONAME libamdhip64.so.7).  Importing it
    # first makes libgrav.so bind to that same runtime, so device pointers and
    # streams from torch are valid in the library (one runtime per process).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_2602_03857_amd/build.py` "
            "(the gravity operators have no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_double)
    P = ctypes.POINTER
    sig = {
        "grav_ctx_opts_default": (None, [P(CtxOpts)]),
        "grav_ctx_create": (ctypes.c_int, [P(vp), P(CtxOpts)]),
        "grav_ctx_destroy": (None, [vp]),
        "grav_last_error": (ctypes.c_char_p, [vp]),
        "grav_workspace_bytes": (u64, [i32, i32, i32, i64, ctypes.c_int, ctypes.c_int, i32]),
        "grav_forward": (ctypes.c_int, [vp, P(CMesh), P(CObs), vp, vp, ctypes.c_int, vp]),
        "grav_adjoint": (ctypes.c_int, [vp, P(CMesh), P(CObs), vp, vp, ctypes.c_int, vp]),
        "grav_dataspace_apply": (ctypes.c_int, [vp, P(CMesh), P(CObs), vp, dbl, vp, vp,
                                                ctypes.c_int, vp]),
        "grav_trace": (ctypes.c_int, [vp, P(CMesh), P(CObs), vp, P(dbl), vp, ctypes.c_int, vp]),
        "grav_trend_surface": (ctypes.c_int, [vp, vp, vp, vp, i64, i32, P(dbl), P(dbl), vp, vp,
                                              vp]),
        "grav_invert": (ctypes.c_int, [vp, P(CMesh), P(CObs), vp, vp, dbl, vp, P(CgOpts), vp, vp,
                                       P(CgInfo), ctypes.c_int, vp]),
        "grav_forward_multi": (ctypes.c_int, [vp, P(CMesh), P(CObs), vp, i32, vp, ctypes.c_int,
                                              vp]),
        "grav_invert_sections": (ctypes.c_int, [vp, P(CMesh), P(CObs), vp, vp, dbl, P(CgOpts),
                                                P(SectionOpts), vp, vp, P(CgInfo), ctypes.c_int,
                                                vp]),
        "grav_forward_static": (ctypes.c_int, [P(CMesh), P(CObs), vp, vp, ctypes.c_int, i32, vp]),
        "grav_server_create": (ctypes.c_int, [P(vp), P(ServerOpts)]),
        "grav_server_submit": (ctypes.c_int, [vp, P(GravRequest), P(ctypes.c_uint64)]),
        "grav_server_poll": (ctypes.c_int, [vp, ctypes.c_uint64, P(i32), P(RequestInfo)]),
        "grav_server_wait": (ctypes.c_int, [vp, ctypes.c_uint64, P(RequestInfo)]),
        "grav_server_cancel": (ctypes.c_int, [vp, ctypes.c_uint64]),
        "grav_server_destroy": (None, [vp]),
        "grav_set_timing": (ctypes.c_int, [vp, i32]),
        "grav_issue_rates": (ctypes.c_int, [vp, P(dbl), vp]),
        "grav_issue_pair_rates": (ctypes.c_int, [vp, P(dbl), vp]),
        "grav_kernel_time": (ctypes.c_int, [vp, ctypes.c_char_p, P(dbl), P(i64)]),
        "grav_reset_timing": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()

EXPORTED = [
    "grav_ctx_opts_default", "grav_ctx_create", "grav_ctx_destroy", "grav_last_error",
    "grav_workspace_bytes", "grav_forward", "grav_adjoint", "grav_dataspace_apply", "grav_trace",
    "grav_trend_surface",
    "grav_invert", "grav_invert_sections", "grav_forward_multi", "grav_forward_static", "grav_set_timing", "grav_kernel_time",
    "grav_reset_timing", "grav_issue_rates", "grav_issue_pair_rates", "grav_server_create", "grav_server_submit", "grav_server_poll",
    "grav_server_wait", "grav_server_cancel", "grav_server_destroy",
]
