"""Process-parallel drivers for the FP64 oracle (row-wise work split over
observations).  TEST INFRASTRUCTURE ONLY.

The arithmetic is exactly ``oracle.prism``'s; this module only distributes
rows over worker processes (fork start method, the problem is inherited).
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from . import prism

_STATE = {}


def _fwd_rows(rows):
    s = _STATE
    return prism.forward(s["mesh"], s["obs"], s["m"], rows=rows)


def _sumsq_rows(rows):
    s = _STATE
    return prism.weighted_row_sumsq(s["mesh"], s["obs"], s["cov"], rows=rows)


def _multi_rows(rows):
    s = _STATE
    return prism.forward_multi(s["mesh"], s["obs"], s["models"], rows=rows)


def _adjoint_rows(rows):
    s = _STATE
    return prism.adjoint(s["mesh"], s["obs"].take(rows), s["v"][rows])[None, :]


def _run(fn, rows, workers, **state):
    rows = np.asarray(rows)
    workers = max(1, min(int(workers), rows.size))
    _STATE.clear()
    _STATE.update(state)
    if workers == 1:
        return fn(rows)
    chunks = np.array_split(rows, workers * 4)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        parts = pool.map(fn, chunks)
    return np.concatenate(parts, axis=0)


def default_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def forward_rows(mesh, obs, m, rows, workers=None):
    """``prism.forward(mesh, obs, m, rows)`` split over processes."""
    return _run(_fwd_rows, rows, workers or default_workers(), mesh=mesh, obs=obs,
                m=np.asarray(m, dtype=np.float64))


def weighted_row_sumsq(mesh, obs, cov, rows, workers=None):
    """``prism.weighted_row_sumsq`` split over processes."""
    return _run(_sumsq_rows, rows, workers or default_workers(), mesh=mesh, obs=obs,
                cov=np.asarray(cov, dtype=np.float64))


def adjoint(mesh, obs, v, rows=None, workers=None):
    """``prism.adjoint`` over the observations ``rows`` (default all): each
    process sums G^T v over its share of the observations, and the shares'
    results are added (G^T v is linear in v)."""
    rows = np.arange(obs.n) if rows is None else np.asarray(rows)
    parts = _run(_adjoint_rows, rows, workers or default_workers(), mesh=mesh, obs=obs,
                 v=np.asarray(v, dtype=np.float64))
    return parts.sum(axis=0)


def forward_multi_rows(mesh, obs, models, rows, workers=None):
    """``prism.forward_multi`` split over processes."""
    return _run(_multi_rows, rows, workers or default_workers(), mesh=mesh, obs=obs,
                models=np.asarray(models, dtype=np.float64))
