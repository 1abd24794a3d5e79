"""Python binding of the continuous-batching server (grav_server_* in
include/grav.h): argument marshalling and lifetime of the request tensors."""
from __future__ import annotations

import ctypes
import threading

import torch

from ._lib import (lib, GravError, GravRequest, RequestInfo, ServerOpts, CgOpts, GRAV_OK,
                   GRAV_ENOCONV, GRAV_ECANCELED)
from .api import DeviceMesh, DeviceObs, _check

REQ_FORWARD, REQ_INVERT = 0, 1


def _info(ri: RequestInfo) -> dict:
    return dict(status=ri.status, iters=ri.iters, relres=ri.relres, lambda_used=ri.lambda_used,
                queue_ms=ri.queue_ms, run_ms=ri.run_ms, state_bytes=ri.state_bytes)


class Server:
    """Continuous-batching server on one device (GRAV_MIXED)."""

    def __init__(self, device: int = 0, max_active: int = 64, budget_bytes: int = 0):
        opts = ServerOpts(device, max_active, budget_bytes)
        h = ctypes.c_void_p()
        rc = lib.grav_server_create(ctypes.byref(h), ctypes.byref(opts))
        if rc != GRAV_OK:
            raise GravError(rc, "grav_server_create failed")
        self._h = h
        self.device = torch.device("cuda", device)
        self._keep = {}          # ticket -> tensors the request reads or writes
        self._lock = threading.Lock()

    def close(self):
        if getattr(self, "_h", None):
            lib.grav_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _stream(self) -> int:
        """torch's current stream on the server's device: the inputs of a
        request are typically produced there, and submit orders the server's
        reads after everything already enqueued on it."""
        return torch.cuda.current_stream(self.device).cuda_stream

    def _submit(self, req: GravRequest, keep) -> int:
        t = ctypes.c_uint64()
        rc = lib.grav_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if rc != GRAV_OK:
            raise GravError(rc, "request rejected")
        with self._lock:
            self._keep[t.value] = keep
        return t.value

    def submit_forward(self, mesh: DeviceMesh, obs: DeviceObs, m, d) -> int:
        _check(m, torch.float64, mesh.ncells, "m", self.device)
        _check(d, torch.float64, obs.n, "d", self.device)
        req = GravRequest(kind=REQ_FORWARD, mesh=mesh.c, obs=obs.c, m=m.data_ptr(), d=d.data_ptr(),
                          stream=self._stream())
        return self._submit(req, (mesh, obs, m, d))

    def submit_invert(self, mesh: DeviceMesh, obs: DeviceObs, d_obs, wdepth, m_out, lam=-1.0,
                      tol=1e-6, max_iter=200, fixed_iters=0) -> int:
        _check(d_obs, torch.float64, obs.n, "d_obs", self.device)
        _check(wdepth, torch.float64, mesh.ncells, "wdepth", self.device)
        _check(m_out, torch.float64, mesh.ncells, "m_out", self.device)
        req = GravRequest(kind=REQ_INVERT, mesh=mesh.c, obs=obs.c, d_obs=d_obs.data_ptr(),
                          wdepth=wdepth.data_ptr(), lam=float(lam),
                          cg=CgOpts(float(tol), int(max_iter), int(fixed_iters), 0, 0, 0, 0, 0, None, None, None),
                          m_out=m_out.data_ptr(), stream=self._stream())
        return self._submit(req, (mesh, obs, d_obs, wdepth, m_out))

    def poll(self, ticket: int):
        done = ctypes.c_int32()
        ri = RequestInfo()
        rc = lib.grav_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(ri))
        if rc != GRAV_OK:
            raise GravError(rc, f"unknown ticket {ticket}")
        if done.value:
            with self._lock:
                self._keep.pop(ticket, None)
            return True, _info(ri)
        return False, None

    def wait(self, ticket: int) -> dict:
        ri = RequestInfo()
        rc = lib.grav_server_wait(self._h, ticket, ctypes.byref(ri))
        with self._lock:
            self._keep.pop(ticket, None)
        if rc not in (GRAV_OK, GRAV_ENOCONV, GRAV_ECANCELED):
            raise GravError(rc, f"request {ticket} failed")
        return _info(ri)

    def cancel(self, ticket: int) -> None:
        """Cancel a queued or running request; it then reports status
        GRAV_ECANCELED through poll / wait (outputs unspecified)."""
        rc = lib.grav_server_cancel(self._h, ticket)
        if rc != GRAV_OK:
            raise GravError(rc, f"unknown ticket {ticket}")
