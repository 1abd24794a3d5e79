"""Write stored FP64 oracle values for the large workloads (tests/golden/*.npz).

Calls only ``oracle`` (and the seeded input generators in ``workloads``).
Run from the repository root:  python tests/golden/make_golden.py [which ...]

Adjoint probes are sign-definite, v = |probe_v|: with v >= 0 the entries of
G^T v are sums over observations without cancellation between them, so a
relative-error bound on them is meaningful (a zero or wrong output fails it).

* paper_scale_rows.npz (178,797 observations x 3,307,500 prisms):
  - rows, d: d = G m at 2,000 seeded observation rows (seed 12345);
  - cells, gtv, gtv_abs, gtv_abs_corners: (G^T v) at 48 seeded cells for
    v = |probe_v|, and the summed magnitudes of the edge terms and of the
    corner terms those entries add up (rounding scales of the two paths);
  - ds_support, ds_v, ds_lambda, ds_rows, ds_out: the data-space operator
    A v = G C G^T v + lambda v (Eq. 10-11) for v supported on 64 seeded
    observations (values |N(0, 1)|, seed 54321), at the 2,000 rows above plus
    the support; lambda = 1e-2 times the mean of the diagonal of G C G^T over
    the support (a sampled form of the trace rule);
  - ds_diag: the diagonal sum_k C_k G_ok^2 at the support rows.
* ellipsoids_100x100x50_rows.npz (10,000 observations x 500,000 prisms):
  - rows, d, cells, gtv, gtv_abs, gtv_abs_corners as above (256 rows, 64
    cells, seed 2222);
  - trace, diag: trace(G C G^T) and its diagonal over all 10,000
    observations, C from the depth weights w = (z + 25 m)^-1;
  - ds_lambda = 1e-2 trace / N and ds_out = A v for v = |probe_v| at every
    observation (the full data-space product).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import inversion, prism, parallel  # noqa: E402
import workloads  # noqa: E402


def _pool_map(fn, args, workers):
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        return pool.starmap(fn, args)


def _cells_parallel(fn, mesh, obs, v, cells, workers):
    chunks = np.array_split(np.asarray(cells), workers)
    return np.concatenate(_pool_map(fn, [(mesh, obs, v, c) for c in chunks], workers))


def _adjoint_checks(mesh, obs, v, cells, workers):
    g = _cells_parallel(prism.adjoint_cells, mesh, obs, v, cells, workers)
    g_abs = _cells_parallel(prism.adjoint_abs_scale, mesh, obs, v, cells, workers)
    g_abs8 = _cells_parallel(prism.adjoint_abs_scale_corners, mesh, obs, v, cells, workers)
    return g, g_abs, g_abs8


def make_paper_scale(workers):
    p = workloads.paper_scale()
    rng = np.random.default_rng(12345)
    rows = np.sort(rng.choice(p.obs.n, 2000, replace=False))
    cells = np.sort(rng.choice(p.mesh.ncells, 48, replace=False))
    t = time.time()
    d = parallel.forward_rows(p.mesh, p.obs, p.m, rows, workers=workers)
    print(f"paper_scale forward rows: {time.time() - t:.1f} s", flush=True)
    t = time.time()
    v = np.abs(p.probe_v)
    g, g_abs, g_abs8 = _adjoint_checks(p.mesh, p.obs, v, cells, workers)
    print(f"paper_scale adjoint cells: {time.time() - t:.1f} s", flush=True)
    # data-space operator for a probe supported on 64 observations
    t = time.time()
    rng_ds = np.random.default_rng(54321)
    support = np.sort(rng_ds.choice(p.obs.n, 64, replace=False))
    v_ds = np.zeros(p.obs.n)
    v_ds[support] = np.abs(rng_ds.standard_normal(support.size))
    cov = inversion.covariance_from_weights(p.wdepth)
    diag = parallel.weighted_row_sumsq(p.mesh, p.obs, cov, support, workers=workers)
    lam = 1e-2 * float(np.mean(diag))
    gt = parallel.adjoint(p.mesh, p.obs, v_ds, rows=support, workers=workers)
    ds_rows = np.union1d(rows, support)
    out = parallel.forward_rows(p.mesh, p.obs, cov * gt, ds_rows, workers=workers) + lam * v_ds[ds_rows]
    print(f"paper_scale data-space rows: {time.time() - t:.1f} s", flush=True)
    np.savez(os.path.join(HERE, "paper_scale_rows.npz"), rows=rows, d=d, cells=cells, gtv=g,
             gtv_abs=g_abs, gtv_abs_corners=g_abs8, ds_support=support, ds_v=v_ds[support],
             ds_lambda=lam, ds_rows=ds_rows, ds_out=out, ds_diag=diag)


def make_ellipsoids(workers):
    p = workloads.ellipsoids_100x100x50()
    rng = np.random.default_rng(2222)
    rows = np.sort(rng.choice(p.obs.n, 256, replace=False))
    cells = np.sort(rng.choice(p.mesh.ncells, 64, replace=False))
    t = time.time()
    d = parallel.forward_rows(p.mesh, p.obs, p.m, rows, workers=workers)
    v = np.abs(p.probe_v)
    g, g_abs, g_abs8 = _adjoint_checks(p.mesh, p.obs, v, cells, workers)
    print(f"ellipsoids_100x100x50 rows and cells: {time.time() - t:.1f} s", flush=True)
    t = time.time()
    cov = inversion.covariance_from_weights(workloads.depth_weights(p.mesh, 25.0))
    diag = parallel.weighted_row_sumsq(p.mesh, p.obs, cov, np.arange(p.obs.n), workers=workers)
    trace = float(diag.sum())
    lam = inversion.lambda_rule(trace, p.obs.n)
    print(f"ellipsoids_100x100x50 trace: {time.time() - t:.1f} s", flush=True)
    t = time.time()
    gt = parallel.adjoint(p.mesh, p.obs, v, workers=workers)
    out = parallel.forward_rows(p.mesh, p.obs, cov * gt, np.arange(p.obs.n), workers=workers) + lam * v
    print(f"ellipsoids_100x100x50 data-space: {time.time() - t:.1f} s", flush=True)
    np.savez(os.path.join(HERE, "ellipsoids_100x100x50_rows.npz"), rows=rows, d=d, cells=cells,
             gtv=g, gtv_abs=g_abs, gtv_abs_corners=g_abs8, trace=trace, diag=diag, ds_lambda=lam,
             ds_out=out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["ellipsoids_100x100x50", "paper_scale"]
    w = parallel.default_workers()
    if "ellipsoids_100x100x50" in which:
        make_ellipsoids(w)
    if "paper_scale" in which:
        make_paper_scale(w)
