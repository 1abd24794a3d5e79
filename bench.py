#!/usr/bin/env python3
"""Benchmark of the matrix-free forward product G m at paper scale on one MI355X.

Workload: 178,797 observations over a 150 x 150 x 147 prism mesh
(3,307,500 prisms, 100 x 100 x 70 m cells), two dykes plus ten random
bodies, synthetic and seeded (``workloads.config4``).  A step is one
``grav_forward`` call in GRAV_MIXED precision: coordinate differences, edge
weights, the forward sweep and the partial-sum reduction, inputs already
resident in HBM.  Metric: prism-observation pairs per second,
pairs = N_obs x N_prisms per step.

Printed (rank 0, one JSON line): the contract fields plus
  roofline      - the forward sweep kernel against the VALU issue limit,
  cpu_baseline  - the FP64 oracle on a bounded sample of rows, on host cores,
  extras        - adjoint sweep, data-space apply, plain-FP64 speed-up, CG
                  iterations/s (a few iterations), error vs the oracle rows.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# Peak VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one lane-slot
# per cycle for a full-rate (non-packed FP32 / FP64) instruction.
PEAK_LANE_SLOTS = 256 * 4 * 16 * 2.4e9
# Algorithmic VALU lane-slots per vertical edge segment of the forward sweep:
# the minimal gfx950 instruction sequence of the edge-segment formula
# (derivation and per-operation table in the design notes).
SLOTS_PER_SEGMENT = 96

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "forward_mixed_config4_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2602_03857_amd", "csrc", f)
                  for f in ("sweeps.hip", "edge_math.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(p, target_s: float, workers: int):
    """FP64 oracle (as it stands) on a bounded sample of config-4 rows."""
    from oracle import parallel
    rng = np.random.default_rng(777)
    rows_probe = rng.choice(p.obs.n, workers, replace=False)
    t0 = time.perf_counter()
    parallel.forward_rows(p.mesh, p.obs, p.m, rows_probe, workers=workers)
    t_probe = time.perf_counter() - t0
    n_rows = int(max(workers, min(4096, workers * max(1, round(target_s / max(t_probe, 1e-3))))))
    rows = rng.choice(p.obs.n, n_rows, replace=False)
    t0 = time.perf_counter()
    parallel.forward_rows(p.mesh, p.obs, p.m, rows, workers=workers)
    dt = time.perf_counter() - t0
    pairs = n_rows * p.mesh.ncells
    return {"value": pairs / dt, "unit": "pairs/s", "cores": workers, "kind": "oracle",
            "sample": f"{n_rows} rows of G m (each over all {p.mesh.ncells} prisms), "
                      f"FP64 NumPy node-shared oracle, {workers} processes, {dt:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cg-iters", type=int, default=3, help="CG iterations timed for it/s")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: --gpus {args.gpus} is not supported "
              "(the library is single-device; multi-GPU sharding is a design note only).",
              file=sys.stderr)
        return 2

    p = workloads.config4()
    n, M = p.obs.n, p.mesh.ncells
    pairs = n * M

    # CPU leg first, before this process touches the GPU (the oracle forks workers).
    cpu = None
    if not args.no_cpu_baseline:
        workers = max(1, min(16, os.cpu_count() or 1))
        cpu = cpu_baseline(p, args.cpu_seconds, workers)
        print(f"[bench] cpu baseline: {cpu['value']:.3e} pairs/s ({cpu['sample']})",
              file=sys.stderr, flush=True)

    lib_path = os.path.join(ROOT, "paper_2602_03857_amd", "libgrav.so")
    if not os.path.exists(lib_path):
        from paper_2602_03857_amd.build import build
        build()
    import torch
    import paper_2602_03857_amd as g

    dev = torch.device("cuda", 0)
    mesh = g.DeviceMesh.from_mesh(p.mesh, dev)
    obs = g.DeviceObs.from_survey(p.obs, dev)
    m = torch.as_tensor(p.m, device=dev)
    d = torch.empty(n, dtype=torch.float64, device=dev)

    # one validated call, then the timed context skips per-call validation
    with g.Context(0, validate=True) as vctx:
        vctx.forward(mesh, obs, m, d, prec=g.GRAV_MIXED)
    torch.cuda.synchronize()
    ctx = g.Context(0, validate=False)
    ctx.set_timing(True)
    for _ in range(args.warmup):
        ctx.forward(mesh, obs, m, d, prec=g.GRAV_MIXED)
    torch.cuda.synchronize()
    ctx.reset_timing()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.forward(mesh, obs, m, d, prec=g.GRAV_MIXED)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    value = pairs * args.steps / dt
    k_ms, k_n = ctx.kernel_time("forward_mixed")
    k_avg_ms = k_ms / max(k_n, 1)
    print(f"[bench] G m: {ms_per_step:.1f} ms/step, sweep kernel {k_avg_ms:.1f} ms avg "
          f"over {k_n} launches, {value:.3e} pairs/s", file=sys.stderr, flush=True)

    segs = (p.mesh.nx + 1) * (p.mesh.ny + 1) * p.mesh.nz
    alg_slots = SLOTS_PER_SEGMENT * segs * n
    achieved = alg_slots / (k_avg_ms * 1e-3)
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("source_hash") == kernel_source_hash():
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_SLOTS / 1e12,
                "unit": "T lane-slots/s", "frac": achieved / PEAK_LANE_SLOTS, "traffic": traffic,
                "kernel": "k_forward_mixed", "kernel_ms": k_avg_ms,
                "slots_per_segment": SLOTS_PER_SEGMENT, "segments_per_launch": segs * n}

    # error vs the oracle on the stored rows
    extras = {}
    gold_path = os.path.join(ROOT, "tests", "golden", "config4_rows.npz")
    if os.path.exists(gold_path):
        gold = np.load(gold_path)
        dn = d.cpu().numpy()[gold["rows"]]
        extras["rel_l2_vs_fp64_oracle_2000_rows"] = float(
            np.linalg.norm(dn - gold["d"]) / np.linalg.norm(gold["d"]))

    if not args.no_extras:
        v = torch.as_tensor(p.probe_v, device=dev)
        gt = torch.empty(M, dtype=torch.float64, device=dev)
        ctx.reset_timing()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.adjoint(mesh, obs, v, gt, prec=g.GRAV_MIXED)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        extras["adjoint_pairs_per_s"] = pairs / t_adj
        extras["adjoint_ms"] = 1e3 * t_adj

        ctx.reset_timing()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.forward(mesh, obs, m, d, prec=g.GRAV_FP64)
        torch.cuda.synchronize()
        t_f64 = time.perf_counter() - t0
        extras["fp64_forward_ms"] = 1e3 * t_f64
        extras["mixed_speedup_over_fp64"] = t_f64 / (ms_per_step * 1e-3)

        w = torch.as_tensor(p.wdepth, device=dev)
        d_obs = d.clone()
        if args.cg_iters > 0:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = ctx.invert(mesh, obs, d_obs, w, lam=1e-12, fixed_iters=args.cg_iters,
                                    prec=g.GRAV_MIXED)
            torch.cuda.synchronize()
            t_cg = time.perf_counter() - t0
            # invert = 1 adjoint (final) + cg_iters x (adjoint + forward)
            per_iter = (t_cg - t_adj) / args.cg_iters
            extras["cg_iterations_per_s"] = 1.0 / per_iter
            extras["cg_seconds_for_50_iterations_est"] = 50 * per_iter
            extras["cg_timed_iterations"] = args.cg_iters

    out = {
        "metric": "prism-obs pairs/s for G.m at 3.3M x 178,797",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded config-4 survey and model)",
        "config": {"workload": "config4: G m, 178,797 obs x 3,307,500 prisms (150x150x147, "
                               "100x100x70 m), GRAV_MIXED",
                   "n_obs": n, "n_prisms": M, "pairs_per_step": pairs},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
