"""Thin Python wrappers over the C ABI: device tensors in, device tensors out.

Each method checks dtypes/devices, passes raw device pointers and the current
torch stream to the library, and raises ``GravError`` on a non-OK status.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import (lib, GravError, CMesh, CObs, CtxOpts, CgOpts, CgInfo, SectionOpts, GRAV_OK,
                   GRAV_ENOCONV, GRAV_MIXED, GRAV_MIXED_BF16X3, GRAV_TREND_SECTION,
                   GRAV_TREND_DOMAIN, OP_FORWARD)


def _device_f64(a, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=torch.float64)
    else:
        t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)
    return t.contiguous()


def _check(t: torch.Tensor, dtype, numel: int, name: str, device) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise TypeError(f"{name} must live on {device}, got {t.device}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


class DeviceMesh:
    """Node coordinate vectors resident on the device (float64, z down)."""

    def __init__(self, xn, yn, zn, device="cuda"):
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.xn = _device_f64(xn, self.device)
        self.yn = _device_f64(yn, self.device)
        self.zn = _device_f64(zn, self.device)
        self.nx, self.ny, self.nz = self.xn.numel() - 1, self.yn.numel() - 1, self.zn.numel() - 1
        self.c = CMesh(self.nx, self.ny, self.nz, self.xn.data_ptr(), self.yn.data_ptr(),
                       self.zn.data_ptr())

    @classmethod
    def from_mesh(cls, mesh, device="cuda") -> "DeviceMesh":
        return cls(mesh.xn, mesh.yn, mesh.zn, device)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz


class DeviceObs:
    """Observation points resident on the device (float64, z down)."""

    def __init__(self, x, y, z, device="cuda"):
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.x = _device_f64(x, self.device)
        self.y = _device_f64(y, self.device)
        self.z = _device_f64(z, self.device)
        self.n = self.x.numel()
        self.c = CObs(self.n, self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr())

    @classmethod
    def from_survey(cls, obs, device="cuda") -> "DeviceObs":
        return cls(obs.x, obs.y, obs.z, device)


def workspace_bytes(nx, ny, nz, n, op=OP_FORWARD, prec=GRAV_MIXED, K=0) -> int:
    return int(lib.grav_workspace_bytes(nx, ny, nz, n, op, prec, K))


def forward_static(mesh: DeviceMesh, obs: DeviceObs, m, d=None, prec=GRAV_MIXED, validate=True,
                   stream=None):
    """d = G m through grav_forward_static (no context; the library's static
    device scratch buffer), on mesh.device.  m: (M,) float64 device tensor."""
    dev = mesh.device
    _check(m, torch.float64, mesh.ncells, "m", dev)
    if d is None:
        d = torch.empty(obs.n, dtype=torch.float64, device=dev)
    _check(d, torch.float64, obs.n, "d", dev)
    with torch.cuda.device(dev):
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        rc = lib.grav_forward_static(ctypes.byref(mesh.c), ctypes.byref(obs.c), m.data_ptr(),
                                     d.data_ptr(), prec, 1 if validate else 0,
                                     ctypes.c_void_p(st.cuda_stream))
    if rc != GRAV_OK:
        raise GravError(rc, lib.grav_last_error(None).decode())
    return d


class Context:
    """A library context: one device, one workspace, one call at a time."""

    def __init__(self, device: int = 0, validate: bool = True, workspace_bytes: int = 0):
        opts = CtxOpts()
        lib.grav_ctx_opts_default(ctypes.byref(opts))
        opts.device = device
        opts.validate = 1 if validate else 0
        opts.workspace_bytes = workspace_bytes
        h = ctypes.c_void_p()
        rc = lib.grav_ctx_create(ctypes.byref(h), ctypes.byref(opts))
        if rc != GRAV_OK:
            raise GravError(rc, lib.grav_last_error(None).decode())
        self._h = h
        self.device = torch.device("cuda", device)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.grav_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def last_error(self) -> str:
        return lib.grav_last_error(self._h).decode()

    def _rc(self, rc: int, allow_noconv: bool = False) -> int:
        if rc == GRAV_OK or (allow_noconv and rc == GRAV_ENOCONV):
            return rc
        raise GravError(rc, self.last_error())

    def _stream(self, stream):
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(stream.cuda_stream)

    # ------------------------------------------------------------ diagnostics
    def set_timing(self, enable: bool = True) -> None:
        self._rc(lib.grav_set_timing(self._h, 1 if enable else 0))

    def kernel_time(self, kernel: str):
        """(total_ms, launches) of a sweep kernel since the last reset (HIP events)."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._rc(lib.grav_kernel_time(self._h, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def reset_timing(self) -> None:
        self._rc(lib.grav_reset_timing(self._h))

    # ------------------------------------------------------------ operators
    def forward(self, mesh: DeviceMesh, obs: DeviceObs, m, d=None, prec=GRAV_MIXED, stream=None):
        """d = G m.  m: (M,) float64 device tensor."""
        _check(m, torch.float64, mesh.ncells, "m", self.device)
        if d is None:
            d = torch.empty(obs.n, dtype=torch.float64, device=self.device)
        _check(d, torch.float64, obs.n, "d", self.device)
        self._rc(lib.grav_forward(self._h, ctypes.byref(mesh.c), ctypes.byref(obs.c),
                                  m.data_ptr(), d.data_ptr(), prec, self._stream(stream)))
        return d

    def adjoint(self, mesh: DeviceMesh, obs: DeviceObs, v, g=None, prec=GRAV_MIXED, stream=None):
        """g = G^T v.  v: (n,) float64 device tensor."""
        _check(v, torch.float64, obs.n, "v", self.device)
        if g is None:
            g = torch.empty(mesh.ncells, dtype=torch.float64, device=self.device)
        _check(g, torch.float64, mesh.ncells, "g", self.device)
        self._rc(lib.grav_adjoint(self._h, ctypes.byref(mesh.c), ctypes.byref(obs.c),
                                  v.data_ptr(), g.data_ptr(), prec, self._stream(stream)))
        return g

    def dataspace_apply(self, mesh, obs, wdepth, lam, v, out=None, prec=GRAV_MIXED, stream=None):
        """out = G diag(wdepth^-2) G^T v + lam v."""
        _check(wdepth, torch.float64, mesh.ncells, "wdepth", self.device)
        _check(v, torch.float64, obs.n, "v", self.device)
        if out is None:
            out = torch.empty(obs.n, dtype=torch.float64, device=self.device)
        _check(out, torch.float64, obs.n, "out", self.device)
        self._rc(lib.grav_dataspace_apply(self._h, ctypes.byref(mesh.c), ctypes.byref(obs.c),
                                          wdepth.data_ptr(), float(lam), v.data_ptr(),
                                          out.data_ptr(), prec, self._stream(stream)))
        return out

    def trace(self, mesh, obs, wdepth, diag=None, prec=GRAV_MIXED, stream=None):
        """trace(G C G^T); fills `diag` (n,) with the per-observation terms if given."""
        _check(wdepth, torch.float64, mesh.ncells, "wdepth", self.device)
        if diag is not None:
            _check(diag, torch.float64, obs.n, "diag", self.device)
        tr = ctypes.c_double()
        self._rc(lib.grav_trace(self._h, ctypes.byref(mesh.c), ctypes.byref(obs.c),
                                wdepth.data_ptr(), ctypes.byref(tr),
                                diag.data_ptr() if diag is not None else None, prec,
                                self._stream(stream)))
        return tr.value

    def issue_rates(self, stream=None):
        """Measured issue rates of the sweeps' instruction classes (chain steps
        per second summed over lanes): fma32, log, rcp, sqrt (each + an FP32
        add), fma64, add32."""
        r = (ctypes.c_double * 6)()
        self._rc(lib.grav_issue_rates(self._h, r, self._stream(stream)))
        return dict(zip(("fma32", "log", "rcp", "sqrt", "fma64", "add32"), list(r)))

    def issue_pair_rates(self, stream=None):
        """Issue rates (chain steps per second summed over lanes) of FP32 FMA
        chains mixed half and half with transcendental or compare-and-select
        chains, on alternating waves and interleaved in every wave."""
        r = (ctypes.c_double * 5)()
        self._rc(lib.grav_issue_pair_rates(self._h, r, self._stream(stream)))
        return dict(zip(("fma_log_alternating", "fma_log_interleaved", "fma_select_alternating",
                         "fma_select_interleaved", "select"), list(r)))

    def trend_surface(self, x, y, v, degree=2, resid=None, trend=None, stream=None):
        """Least-squares trend surface of `degree` (1 or 2) through (x, y, v)
        (device float64 vectors of one length).  Returns (coef[6], frame
        (x0, y0, L)) and fills `resid` (v - T) and/or `trend` (T) if given."""
        n = v.numel()
        for t, name in ((x, "x"), (y, "y"), (v, "v")):
            _check(t, torch.float64, n, name, self.device)
        for t, name in ((resid, "resid"), (trend, "trend")):
            if t is not None:
                _check(t, torch.float64, n, name, self.device)
        coef = (ctypes.c_double * 6)()
        frame = (ctypes.c_double * 3)()
        self._rc(lib.grav_trend_surface(self._h, x.data_ptr(), y.data_ptr(), v.data_ptr(), n,
                                        int(degree), coef, frame,
                                        resid.data_ptr() if resid is not None else None,
                                        trend.data_ptr() if trend is not None else None,
                                        self._stream(stream)))
        return list(coef), tuple(frame)

    def invert(self, mesh, obs, d_obs, wdepth, lam=-1.0, m_ref=None, tol=1e-6, max_iter=200,
               fixed_iters=0, m_out=None, d_pred=None, want_pred=False, prec=GRAV_MIXED,
               stream=None, precond=0, restart=0, max_cycles=30, max_halvings=5,
               history_cap=0, y0=None, y_out=None, graph=False):
        """Data-space CG inversion (Eq. 11).  Returns (m, d_pred or None, info dict).

        restart > 0 selects the restarted policy (cycles of at most `restart`
        CG iterations, at most `max_cycles` cycles, step backtracking with at
        most `max_halvings` halvings per cycle); max_iter is then unused.
        history_cap > 0 returns the misfit log (relative residual after each
        CG iteration, at most history_cap entries) as info["history"].
        y0 (n,) starts CG from that data-space iterate (warm start / resume);
        y_out (n,) receives the final iterate.  graph=True replays each plain
        or Jacobi CG iteration from a HIP graph captured once per solve."""
        _check(d_obs, torch.float64, obs.n, "d_obs", self.device)
        _check(wdepth, torch.float64, mesh.ncells, "wdepth", self.device)
        if m_ref is not None:
            _check(m_ref, torch.float64, mesh.ncells, "m_ref", self.device)
        if m_out is None:
            m_out = torch.empty(mesh.ncells, dtype=torch.float64, device=self.device)
        _check(m_out, torch.float64, mesh.ncells, "m_out", self.device)
        if d_pred is None and want_pred:
            d_pred = torch.empty(obs.n, dtype=torch.float64, device=self.device)
        if d_pred is not None:
            _check(d_pred, torch.float64, obs.n, "d_pred", self.device)
        for t, name in ((y0, "y0"), (y_out, "y_out")):
            if t is not None:
                _check(t, torch.float64, obs.n, name, self.device)
        hist = (ctypes.c_double * max(int(history_cap), 1))()
        cg = CgOpts(float(tol), int(max_iter), int(fixed_iters), int(precond), int(restart),
                    int(max_cycles), int(max_halvings), int(history_cap),
                    ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)) if history_cap > 0 else None,
                    y0.data_ptr() if y0 is not None else None,
                    y_out.data_ptr() if y_out is not None else None, int(bool(graph)))
        info = CgInfo()
        rc = lib.grav_invert(self._h, ctypes.byref(mesh.c), ctypes.byref(obs.c), d_obs.data_ptr(),
                             wdepth.data_ptr(), float(lam),
                             m_ref.data_ptr() if m_ref is not None else None, ctypes.byref(cg),
                             m_out.data_ptr(), d_pred.data_ptr() if d_pred is not None else None,
                             ctypes.byref(info), prec, self._stream(stream))
        self._rc(rc, allow_noconv=True)
        return m_out, d_pred, dict(iters=info.iters, relres=info.relres,
                                   lambda_used=info.lambda_used, trace=info.trace,
                                   cycles=info.cycles, halvings=info.halvings,
                                   history=(list(hist[:min(info.iters, history_cap)])
                                            if history_cap > 0 and not fixed_iters else None),
                                   converged=(rc == GRAV_OK))

    def invert_sections(self, mesh, obs, d_obs, wdepth, ysplit, data_degree=2,
                        data_scope="section", model_degree=2, lam=-1.0, tol=1e-6, max_iter=200,
                        fixed_iters=0, precond=0, restart=0, max_cycles=30, max_halvings=5,
                        m_out=None, m_detrended=None, detrend=True, prec=GRAV_MIXED,
                        stream=None, graph=False):
        """Regional inversion by adjoining sections along y (split at the mesh
        node rows `ysplit`, 0 ... ny), each inverted on its own, combined, and
        (detrend) a per-layer trend surface of `model_degree` removed.
        data_scope: "section" or "domain".  Returns (m_out, m_detrended or
        None, list of per-section info dicts)."""
        _check(d_obs, torch.float64, obs.n, "d_obs", self.device)
        _check(wdepth, torch.float64, mesh.ncells, "wdepth", self.device)
        if m_out is None:
            m_out = torch.empty(mesh.ncells, dtype=torch.float64, device=self.device)
        _check(m_out, torch.float64, mesh.ncells, "m_out", self.device)
        if m_detrended is None and detrend:
            m_detrended = torch.empty(mesh.ncells, dtype=torch.float64, device=self.device)
        if m_detrended is not None:
            _check(m_detrended, torch.float64, mesh.ncells, "m_detrended", self.device)
        scope = {"section": GRAV_TREND_SECTION, "domain": GRAV_TREND_DOMAIN}[data_scope]
        nsec = len(ysplit) - 1
        split = (ctypes.c_int32 * len(ysplit))(*[int(j) for j in ysplit])
        so = SectionOpts(nsec, ctypes.cast(split, ctypes.POINTER(ctypes.c_int32)), int(data_degree),
                         scope, int(model_degree))
        cg = CgOpts(float(tol), int(max_iter), int(fixed_iters), int(precond), int(restart),
                    int(max_cycles), int(max_halvings), 0, None, None, None, int(bool(graph)))
        infos = (CgInfo * max(nsec, 1))()
        rc = lib.grav_invert_sections(self._h, ctypes.byref(mesh.c), ctypes.byref(obs.c),
                                      d_obs.data_ptr(), wdepth.data_ptr(), float(lam),
                                      ctypes.byref(cg), ctypes.byref(so), m_out.data_ptr(),
                                      m_detrended.data_ptr() if m_detrended is not None else None,
                                      infos, prec, self._stream(stream))
        self._rc(rc, allow_noconv=True)
        return m_out, m_detrended, [dict(iters=i.iters, relres=i.relres, lambda_used=i.lambda_used,
                                         trace=i.trace, cycles=i.cycles, halvings=i.halvings)
                                    for i in infos[:nsec]]

    def forward_multi(self, mesh, obs, models, D=None, prec=GRAV_MIXED_BF16X3, stream=None):
        """D = G M for models (M, K) float32 (model index fastest); returns (n, K) float32."""
        if models.dim() != 2:
            raise ValueError("models must be (M, K)")
        K = models.shape[1]
        _check(models, torch.float32, mesh.ncells * K, "models", self.device)
        if D is None:
            D = torch.empty((obs.n, K), dtype=torch.float32, device=self.device)
        _check(D, torch.float32, obs.n * K, "D", self.device)
        self._rc(lib.grav_forward_multi(self._h, ctypes.byref(mesh.c), ctypes.byref(obs.c),
                                        models.data_ptr(), K, D.data_ptr(), prec,
                                        self._stream(stream)))
        return D
