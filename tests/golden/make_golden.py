"""Write stored FP64 oracle values for the large workloads (tests/golden/*.npz).

Calls only ``oracle`` (and the seeded input generators in ``workloads``).
Run from the repository root:  python tests/golden/make_golden.py [which ...]

* paper_scale_rows.npz : d = G m at 2,000 seeded observation rows of the
  178,797 x 3,307,500 paper-scale workload (seed 12345 picks the rows),
  (G^T v) at 48 seeded cells for the workload's probe vector v, and the
  absolute term scale of those cells (tolerance of the FP32 edge terms).
* ellipsoids_100x100x50_rows.npz : the same at 256 rows and 64 cells of the 10,000 x
  500,000 forward/adjoint workload, plus the corner-term scale (tolerance of
  the FP64 node evaluation).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import prism, parallel  # noqa: E402
import workloads  # noqa: E402


def _adjoint_cells_parallel(mesh, obs, v, cells, workers):
    import multiprocessing as mp
    chunks = np.array_split(np.asarray(cells), workers)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        parts = pool.starmap(prism.adjoint_cells, [(mesh, obs, v, c) for c in chunks])
    return np.concatenate(parts)


def make_paper_scale(workers):
    p = workloads.paper_scale()
    rng = np.random.default_rng(12345)
    rows = np.sort(rng.choice(p.obs.n, 2000, replace=False))
    cells = np.sort(rng.choice(p.mesh.ncells, 48, replace=False))
    t = time.time()
    d = parallel.forward_rows(p.mesh, p.obs, p.m, rows, workers=workers)
    print(f"paper_scale rows: {time.time() - t:.1f} s", flush=True)
    t = time.time()
    g = _adjoint_cells_parallel(p.mesh, p.obs, p.probe_v, cells, workers)
    g_abs = prism.adjoint_abs_scale(p.mesh, p.obs, p.probe_v, cells)
    print(f"paper_scale cells: {time.time() - t:.1f} s", flush=True)
    np.savez(os.path.join(HERE, "paper_scale_rows.npz"), rows=rows, d=d, cells=cells, gtv=g,
             gtv_abs=g_abs)


def make_ellipsoids(workers):
    p = workloads.ellipsoids_100x100x50()
    rng = np.random.default_rng(2222)
    rows = np.sort(rng.choice(p.obs.n, 256, replace=False))
    cells = np.sort(rng.choice(p.mesh.ncells, 64, replace=False))
    t = time.time()
    d = parallel.forward_rows(p.mesh, p.obs, p.m, rows, workers=workers)
    g = _adjoint_cells_parallel(p.mesh, p.obs, p.probe_v, cells, workers)
    g_abs = prism.adjoint_abs_scale(p.mesh, p.obs, p.probe_v, cells)
    g_abs8 = prism.adjoint_abs_scale_corners(p.mesh, p.obs, p.probe_v, cells)
    print(f"ellipsoids_100x100x50: {time.time() - t:.1f} s", flush=True)
    np.savez(os.path.join(HERE, "ellipsoids_100x100x50_rows.npz"), rows=rows, d=d, cells=cells, gtv=g,
             gtv_abs=g_abs, gtv_abs_corners=g_abs8)


if __name__ == "__main__":
    which = sys.argv[1:] or ["ellipsoids_100x100x50", "paper_scale"]
    w = parallel.default_workers()
    if "ellipsoids_100x100x50" in which:
        make_ellipsoids(w)
    if "paper_scale" in which:
        make_paper_scale(w)
