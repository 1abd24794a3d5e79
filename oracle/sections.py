"""FP64 CPU oracle for the regional section workflow (paper Section 4.5, with
the residual separation of Section 2.2).

TEST INFRASTRUCTURE ONLY (see ``oracle.prism``).  Plain NumPy FP64.

The workflow, in the paper's order:

1. Residual separation (Section 2.2): the regional component of the data is
   removed with a least-squares polynomial trend surface in the station
   coordinates (second degree in the paper); the residual is the input of the
   inversion.
2. Sections (Section 4.5): a regional problem too large to invert at once is
   divided into adjoining sections, each inverted on its own (Eq. 11) with its
   own stations.
3. The section models are combined into one regional model.
4. A single polynomial trend surface is fitted across the complete domain
   to the combined model and removed, which evens out the differences the
   independent section inversions leave at their boundaries.

Readings where the paper is not explicit (each is a parameter here):

* Sections adjoin along y, split at mesh node indices ``ysplit``
  (0 = ysplit[0] < ... < ysplit[-1] = ny); station o belongs to the last
  section s whose lower boundary yn[ysplit[s]] is <= y_o (section 0 for
  stations below the first boundary), so every station is in exactly one
  section and a station on a boundary goes to the section above it.
* The data trend of step 1 is fitted per section (``data_scope="section"``:
  each section is processed like a survey of its own, which is what leaves
  the boundary differences step 4 addresses) or once over all stations
  (``data_scope="domain"``); degree 0 skips it.
* The trend surface of step 4 is fitted layer by layer, to the cell values of
  each layer of the combined model at the cell-centre (x, y), and subtracted;
  degree 0 skips it.
* lambda < 0 selects each section's own 1e-2 trace(G C G^T) / N_s.
"""
from __future__ import annotations

import numpy as np

from . import inversion, prism, trend


def section_of_stations(mesh, obs, ysplit) -> np.ndarray:
    """Section index of every station (the assignment rule above)."""
    ysplit = np.asarray(ysplit)
    bounds = mesh.yn[ysplit[1:-1]]                  # interior boundaries
    return np.searchsorted(bounds, obs.y, side="right")


def sub_mesh(mesh, j0, j1):
    """The section's mesh: node rows j0 .. j1 of y (cells j0 .. j1 - 1)."""
    return type(mesh)(mesh.xn, mesh.yn[j0:j1 + 1], mesh.zn)


def cell_slice(mesh, j0, j1) -> np.ndarray:
    """Flat regional cell indices of the section's cells, in the section
    mesh's own cell order (i, j - j0, k)."""
    idx = np.arange(mesh.ncells).reshape(mesh.shape)
    return idx[:, j0:j1, :].reshape(-1)


def model_trend_residual(mesh, m, degree):
    """Step 4: per layer k, the model minus its least-squares trend surface
    of the given degree over the cell centres (x, y)."""
    mm = np.asarray(m, dtype=np.float64).reshape(mesh.shape)
    if degree == 0:
        return mm.reshape(-1).copy()
    xc = 0.5 * (mesh.xn[:-1] + mesh.xn[1:])
    yc = 0.5 * (mesh.yn[:-1] + mesh.yn[1:])
    X, Y = np.meshgrid(xc, yc, indexing="ij")
    out = np.empty_like(mm)
    for k in range(mesh.nz):
        _, r = trend.trend_surface(X.reshape(-1), Y.reshape(-1), mm[:, :, k].reshape(-1), degree)
        out[:, :, k] = r.reshape(mesh.nx, mesh.ny)
    return out.reshape(-1)


def invert_sections(mesh, obs, d_obs, wdepth, ysplit, data_degree=2, data_scope="section",
                    model_degree=2, lam=-1.0):
    """Steps 1-4 with dense Cholesky solves of Eq. 11 per section (tiny
    sections only).  Returns (combined model, combined model minus its
    per-layer trend, list of per-section dicts)."""
    d_obs = np.asarray(d_obs, dtype=np.float64)
    wdepth = np.asarray(wdepth, dtype=np.float64)
    sec = section_of_stations(mesh, obs, ysplit)
    d_in = d_obs.copy()
    if data_degree and data_scope == "domain":
        _, d_in = trend.trend_surface(obs.x, obs.y, d_obs, data_degree)
    m = np.zeros(mesh.ncells)
    info = []
    for s in range(len(ysplit) - 1):
        j0, j1 = int(ysplit[s]), int(ysplit[s + 1])
        rows = np.flatnonzero(sec == s)
        sm = sub_mesh(mesh, j0, j1)
        so = obs.take(rows)
        ds = d_in[rows]
        if data_degree and data_scope == "section":
            _, ds = trend.trend_surface(so.x, so.y, ds, data_degree)
        cells = cell_slice(mesh, j0, j1)
        cov = inversion.covariance_from_weights(wdepth[cells])
        G = np.stack([prism.sensitivity_row(sm, so.x[o], so.y[o], so.z[o]) for o in range(so.n)])
        lam_s = lam
        trace = float(np.einsum("ok,k,ok->", G, cov, G))
        if lam_s < 0:
            lam_s = inversion.lambda_rule(trace, so.n)
        ms, _ = inversion.invert_dense(G, cov, lam_s, ds)
        m[cells] = ms
        info.append(dict(rows=rows, lam=lam_s, trace=trace, d_in=ds))
    return m, model_trend_residual(mesh, m, model_degree), info
