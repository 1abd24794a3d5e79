"""Python binding of the MI355X prism-gravity library (``libgrav.so``).

Argument marshalling only: every step of every operator runs in the HIP
kernels behind the C ABI declared in ``include/grav.h``.  PyTorch provides
device memory and streams.  Importing this module loads the in-tree
``libgrav.so`` and raises ``ImportError`` when it has not been built
(``python paper_2602_03857_amd/build.py``); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

from ._lib import (  # noqa: F401
    LIB_PATH, lib, GravError, GRAV_OK, GRAV_EINVAL, GRAV_ENOMEM, GRAV_EDEVICE, GRAV_ENOCONV,
    GRAV_EBUSY, GRAV_ECANCELED, GRAV_FP64, GRAV_MIXED, GRAV_MIXED_BF16X3, GRAV_FP32_VALU, GRAV_GAMMA,
    GRAV_STATIC_SCRATCH_BYTES,
    OP_FORWARD, OP_ADJOINT, OP_DATASPACE, OP_TRACE, OP_INVERT, OP_FORWARD_MULTI, OP_TREND,
    OP_SECTIONS, GRAV_TREND_SECTION, GRAV_TREND_DOMAIN,
    CMesh, CObs, CtxOpts, CgOpts, CgInfo,
)
from .api import Context, DeviceMesh, DeviceObs, forward_static, workspace_bytes  # noqa: F401
from .serve import Server  # noqa: F401

__all__ = ["Context", "Server", "DeviceMesh", "DeviceObs", "forward_static", "workspace_bytes",
           "GravError", "lib",
           "GRAV_FP64", "GRAV_MIXED", "GRAV_MIXED_BF16X3", "GRAV_FP32_VALU", "GRAV_GAMMA"]
