#!/usr/bin/env python3
"""Benchmark of the matrix-free forward product G m at paper scale on one MI355X.

Workload: 178,797 observations over a 150 x 150 x 147 prism mesh
(3,307,500 prisms, 100 x 100 x 70 m cells), two dykes plus ten random
bodies, synthetic and seeded (``workloads.paper_scale``).  A step is one
``grav_forward`` call in GRAV_MIXED precision: coordinate differences, edge
weights, the forward sweep and the partial-sum reduction, inputs already
resident in HBM.  Metric: prism-observation pairs per second,
pairs = N_obs x N_prisms per step.

Printed (rank 0, one JSON line): the contract fields plus
  roofline      - the forward sweep kernel against the VALU issue limit,
  cpu_baseline  - the FP64 oracle on a bounded sample of rows, on host cores,
  extras        - adjoint sweep, data-space apply, plain-FP64 speed-up, CG
                  iterations/s (a few iterations), error vs the oracle rows,
                  and (serving) CG solve p50/p99 latency over the first 60
                  requests of the serving stream with an FP64 FIFO baseline.
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

# Roofline of the sweeps (instruction-issue-bound kernels).
# Peak: MI355X FP32 vector 157.3 TFLOP/s = 78.65e12 full-rate lane operations
# per second (FMA = one operation).  Algorithmic cost of one (observation,
# vertical edge segment) pair: the minimal gfx950 instruction sequence of the
# edge-segment formula (per-operation table in the design notes), 94
# instructions (6 transcendental: 1 sqrt, 3 rcp, 2 log) for layers near the
# top, and for "deep" layers (top at least 9 thicknesses and 1 mm below the
# mesh top, where the atan difference needs no range reduction, no limit
# select is needed and the log1p arguments stay below 1/4) 58 in the forward
# and 56 in the adjoint (5 transcendental): there atan(u2) is carried down the
# column by the atan addition formula, one FP64 add with two conversions in
# the forward and one FP32 add in the adjoint's walks of at most 16 layers,
# instead of a range-reduced atan.  Every walk down deep layers starts its
# angle with one range-reduced atan (17 instructions, 1 transcendental): once
# per (observation, column) in the forward and once per (observation, column,
# deep layer chunk) in the adjoint.  Issue cost relative to an FP32 add,
# measured with --issue-probe (dependent chains of one instruction class): a
# transcendental takes 2 slots, an FP64 instruction 1; issue slots =
# instructions + transcendentals * (2 - 1).
PEAK_SLOTS = 157.3e12 / 2.0
INSTR_SHALLOW, TRANS_SHALLOW = 94, 6
INSTR_DEEP_FWD, INSTR_DEEP_ADJ, TRANS_DEEP = 58, 56, 5
INSTR_ANCHOR, TRANS_ANCHOR = 17, 1
TRANS_COST, FP64_COST = 2, 1
ADJ_LAYERS = 16          # layers per lane in the mixed adjoint (chunk plan below)
DEEP_RATIO = 9.0
DEEP_MIN_DEPTH = 1e-3


def slots(instr: int, trans: int) -> int:
    return instr + trans * (TRANS_COST - 1)


def adjoint_deep_chunks(nz: int, kdeep: int) -> int:
    """Layer chunks of the mixed adjoint over the deep layers (the library's
    plan chunks the layers above the first deep one and the deep ones
    separately, at most 16 layers a chunk)."""
    return -(-(nz - kdeep) // ADJ_LAYERS)


def sweep_costs(n: int, ncols: int, nz: int, kdeep: int):
    """(instructions, issue slots) per launch of the forward and of the adjoint."""
    ndeep = nz - kdeep
    fwd_i = kdeep * INSTR_SHALLOW + ndeep * INSTR_DEEP_FWD + (INSTR_ANCHOR if ndeep else 0)
    fwd_s = (kdeep * slots(INSTR_SHALLOW, TRANS_SHALLOW) + ndeep * slots(INSTR_DEEP_FWD, TRANS_DEEP)
             + (slots(INSTR_ANCHOR, TRANS_ANCHOR) if ndeep else 0))
    nch = adjoint_deep_chunks(nz, kdeep)
    adj_i = kdeep * INSTR_SHALLOW + ndeep * INSTR_DEEP_ADJ + nch * INSTR_ANCHOR
    adj_s = (kdeep * slots(INSTR_SHALLOW, TRANS_SHALLOW) + ndeep * slots(INSTR_DEEP_ADJ, TRANS_DEEP)
             + nch * slots(INSTR_ANCHOR, TRANS_ANCHOR))
    k = n * ncols
    return {"fwd": (k * fwd_i, k * fwd_s), "adj": (k * adj_i, k * adj_s)}


def first_deep_layer(zn) -> int:
    """Same rule as the library: every layer from this index on has its top at
    least DEEP_RATIO thicknesses and DEEP_MIN_DEPTH below the mesh top."""
    k = len(zn) - 1
    while (k > 0 and (zn[k - 1] - zn[0]) >= DEEP_RATIO * (zn[k] - zn[k - 1])
           and (zn[k - 1] - zn[0]) >= DEEP_MIN_DEPTH):
        k -= 1
    return k


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "forward_mixed_paper_scale_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2602_03857_amd", "csrc", f)
                  for f in ("sweeps.hip", "sweep_bodies.h", "edge_math.h", "grav_internal.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(p, target_s: float, workers: int):
    """FP64 oracle (as it stands) on a bounded sample of the paper-scale rows: batches
    of seeded rows until about target_s seconds of wall time."""
    from oracle import parallel
    rng = np.random.default_rng(777)
    order = rng.permutation(p.obs.n)
    batch = 8 * workers
    done, dt = 0, 0.0
    while dt < target_s and done + batch <= p.obs.n:
        rows = order[done:done + batch]
        t0 = time.perf_counter()
        parallel.forward_rows(p.mesh, p.obs, p.m, rows, workers=workers)
        dt += time.perf_counter() - t0
        done += batch
    pairs = done * p.mesh.ncells
    return {"value": pairs / dt, "unit": "pairs/s", "cores": workers, "kind": "oracle",
            "sample": f"{done} seeded rows of G m (each over all {p.mesh.ncells} prisms), "
                      f"FP64 NumPy node-shared oracle, {workers} processes, {dt:.1f} s"}


def multi_model_extras(g, torch, dev):
    """64 density models on the 500k-cell mesh with 10,000 observations:
    split-bf16 MFMA and FP32-VALU contractions against 64 single forwards."""
    p3 = workloads.ellipsoids_100x100x50()
    models = workloads.smoothed_box_models(p3.mesh).astype(np.float32)
    mesh = g.DeviceMesh.from_mesh(p3.mesh, dev)
    obs = g.DeviceObs.from_survey(p3.obs, dev)
    mt = torch.as_tensor(models, device=dev)
    D = torch.empty((p3.obs.n, models.shape[1]), dtype=torch.float32, device=dev)
    ctx = g.Context(0, validate=False)
    ctx.set_timing(True)
    res = {}
    for prec, key in ((g.GRAV_MIXED_BF16X3, "multi_bf16x3"), (g.GRAV_FP32_VALU, "multi_fp32")):
        ctx.forward_multi(mesh, obs, mt, D, prec=prec)
        torch.cuda.synchronize()
        ctx.reset_timing()
        for _ in range(2):
            ctx.forward_multi(mesh, obs, mt, D, prec=prec)
        torch.cuda.synchronize()
        ms, nl = ctx.kernel_time(key)
        res[key + "_kernel_ms"] = ms / nl
    m1 = torch.as_tensor(models[:, 0].astype(np.float64), device=dev)
    d1 = torch.empty(p3.obs.n, dtype=torch.float64, device=dev)
    ctx.forward(mesh, obs, m1, d1, prec=g.GRAV_MIXED)
    torch.cuda.synchronize()
    ctx.reset_timing()
    for _ in range(3):
        ctx.forward(mesh, obs, m1, d1, prec=g.GRAV_MIXED)
    torch.cuda.synchronize()
    ms, nl = ctx.kernel_time("forward_mixed")
    single = ms / nl
    pairs = p3.obs.n * p3.mesh.ncells * models.shape[1]
    res["single_forward_kernel_ms"] = single
    res["multi_speedup_vs_64_single_forwards"] = 64 * single / res["multi_bf16x3_kernel_ms"]
    res["multi_bf16x3_model_pairs_per_s"] = pairs / (res["multi_bf16x3_kernel_ms"] * 1e-3)
    ctx.close()
    return res


def ellipsoids_extras(g, torch, dev):
    """The 10,000-observation x 500,000-prism forward/adjoint workload in both
    precisions: kernel times and errors on the stored FP64 oracle rows/cells."""
    p = workloads.ellipsoids_100x100x50()
    mesh = g.DeviceMesh.from_mesh(p.mesh, dev)
    obs = g.DeviceObs.from_survey(p.obs, dev)
    m = torch.as_tensor(p.m, device=dev)
    # the stored G^T v cells are for the sign-definite probe |probe_v|
    v = torch.as_tensor(np.abs(p.probe_v), device=dev)
    gold_path = os.path.join(ROOT, "tests", "golden", "ellipsoids_100x100x50_rows.npz")
    gold = np.load(gold_path) if os.path.exists(gold_path) else None
    ctx = g.Context(0, validate=False)
    ctx.set_timing(True)
    res = {}
    for prec, tag in ((g.GRAV_MIXED, "mixed"), (g.GRAV_FP64, "f64")):
        d = ctx.forward(mesh, obs, m, prec=prec)
        gt = ctx.adjoint(mesh, obs, v, prec=prec)
        torch.cuda.synchronize()
        ctx.reset_timing()
        for _ in range(3):
            ctx.forward(mesh, obs, m, d, prec=prec)
            ctx.adjoint(mesh, obs, v, gt, prec=prec)
        torch.cuda.synchronize()
        fms, fn = ctx.kernel_time("forward_" + tag)
        ams, an = ctx.kernel_time("adjoint_" + tag)
        res[f"ellipsoids_forward_{tag}_kernel_ms"] = fms / fn
        res[f"ellipsoids_adjoint_{tag}_kernel_ms"] = ams / an
        if gold is not None:
            dn = d.cpu().numpy()[gold["rows"]]
            res[f"ellipsoids_forward_{tag}_rel_l2"] = float(
                np.linalg.norm(dn - gold["d"]) / np.linalg.norm(gold["d"]))
            gn = gt.cpu().numpy()[gold["cells"]]
            res[f"ellipsoids_adjoint_{tag}_rel_l2"] = float(
                np.linalg.norm(gn - gold["gtv"]) / np.linalg.norm(gold["gtv"]))
    ctx.close()
    return res


def _serve_inputs(g, torch, dev, reqs, ctx):
    """Materialise the request stream on the device (not timed): meshes,
    surveys, models; noisy data for inversions (d_clean from the library)."""
    out = []
    for r in reqs:
        p = r["build"]()
        mesh = g.DeviceMesh.from_mesh(p.mesh, dev)
        obs = g.DeviceObs.from_survey(p.obs, dev)
        item = dict(t=r["t"], kind=r["kind"], mesh=mesh, obs=obs, n=p.obs.n, M=p.mesh.ncells)
        m = torch.as_tensor(p.m, device=dev)
        if r["kind"] == "forward":
            item.update(m=m, d=torch.empty(p.obs.n, dtype=torch.float64, device=dev))
        else:
            d_clean = ctx.forward(mesh, obs, m, prec=g.GRAV_MIXED)
            rms = torch.sqrt(torch.mean(d_clean * d_clean))
            d_obs = d_clean + p.noise_level * rms * torch.as_tensor(p.noise_draws, device=dev)
            item.update(d_obs=d_obs.contiguous(), w=torch.as_tensor(p.wdepth, device=dev),
                        m_out=torch.empty(p.mesh.ncells, dtype=torch.float64, device=dev),
                        tol=p.cg_tol, max_iter=p.cg_iters)
        out.append(item)
    torch.cuda.synchronize()
    return out


def _percentiles(lat):
    lat = np.sort(np.asarray(lat))
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def serve_replay(g, torch, dev, n_requests, max_active, budget_gb, fifo_requests,
                 fifo_budget_s=None, progress=True):
    """Replay the first n_requests of the serving stream (Poisson arrivals)
    open-loop on wall-clock time through the continuous-batching server, then
    the first fifo_requests of the same arrivals through a one-at-a-time FIFO
    of the plain FP64 single-call path (stopped after fifo_budget_s seconds of
    wall time if given; the requests it finished are reported)."""
    from paper_2602_03857_amd import GRAV_ENOCONV
    reqs = workloads.serving_stream()[:n_requests]
    ctx = g.Context(0, validate=False)
    items = _serve_inputs(g, torch, dev, reqs, ctx)
    pairs = [it["n"] * it["M"] for it in items]
    if progress:
        print(f"[serve] {len(items)} requests staged on the device", file=sys.stderr, flush=True)

    # continuous batching
    lat, iters, noconv = [None] * len(items), {}, 0
    srv = g.Server(0, max_active=max_active, budget_bytes=budget_gb << 30)
    t0 = time.perf_counter()
    pending, nxt = {}, 0
    while nxt < len(items) or pending:
        now = time.perf_counter() - t0
        while nxt < len(items) and items[nxt]["t"] <= now:
            it = items[nxt]
            if it["kind"] == "forward":
                tk = srv.submit_forward(it["mesh"], it["obs"], it["m"], it["d"])
            else:
                tk = srv.submit_invert(it["mesh"], it["obs"], it["d_obs"], it["w"], it["m_out"],
                                       lam=-1.0, tol=it["tol"], max_iter=it["max_iter"])
            pending[tk] = nxt
            nxt += 1
        for tk in list(pending):
            done, info = srv.poll(tk)
            if done:
                k = pending.pop(tk)
                it = items[k]
                _ = (it["d"] if it["kind"] == "forward" else it["m_out"]).cpu()
                lat[k] = time.perf_counter() - t0 - it["t"]
                if it["kind"] != "forward":
                    iters[k] = info["iters"]
                    noconv += int(info["status"] == GRAV_ENOCONV)
                ndone = sum(x is not None for x in lat)
                if progress and ndone % 20 == 0:
                    print(f"[serve] {ndone} done", file=sys.stderr, flush=True)
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    srv.close()
    p50, p99 = _percentiles(lat)
    inv = [lat[i] for i, it in enumerate(items) if it["kind"] != "forward"]
    i50, i99 = _percentiles(inv) if inv else (0.0, 0.0)
    # segment pairs swept: forward = 1 sweep; inversion = trace (2) + 2 per CG iteration + final adjoint
    served_pairs = sum(pairs[i] if it["kind"] == "forward" else pairs[i] * (2 * iters[i] + 3)
                       for i, it in enumerate(items))
    res = {"workload": f"serving_stream: first {len(items)} of 200 requests (Poisson arrivals, "
                       "mean gap 0.5 s; forward or inversion, N 1k-40k, 50k-800k cells; "
                       "CG to 1e-6, at most 200 iterations), GRAV_MIXED",
           "requests": len(items), "p50_s": p50, "p99_s": p99, "inversion_p50_s": i50,
           "inversion_p99_s": i99, "inversions": len(inv),
           "inversions_at_iteration_cap": noconv, "wall_s": wall,
           "requests_per_s": len(items) / wall,
           "served_segment_pairs_per_s": served_pairs / wall,
           "pairs_per_s_forward_requests": sum(pairs[i] for i, it in enumerate(items)
                                               if it["kind"] == "forward") / wall,
           "mean_cg_iters": float(np.mean(list(iters.values()))) if iters else 0}

    # error of every served forward result against the plain FP64 path
    errs = []
    for it in items:
        if it["kind"] == "forward":
            ref = ctx.forward(it["mesh"], it["obs"], it["m"], prec=g.GRAV_FP64)
            errs.append(float(torch.linalg.norm(it["d"] - ref) / torch.linalg.norm(ref)))
    if errs:
        res["forward_rel_l2_vs_fp64"] = {"requests": len(errs), "max": max(errs),
                                         "median": float(np.median(errs))}

    # one-at-a-time FIFO of the plain FP64 path on the same arrivals
    nb = min(fifo_requests, len(items))
    if nb > 0:
        ctx64 = g.Context(0, validate=False)
        lat_b = []
        t0 = time.perf_counter()
        for it in items[:nb]:
            now = time.perf_counter() - t0
            if fifo_budget_s is not None and now > fifo_budget_s:
                break
            if now < it["t"]:
                time.sleep(it["t"] - now)
            if it["kind"] == "forward":
                ctx64.forward(it["mesh"], it["obs"], it["m"], it["d"], prec=g.GRAV_FP64)
                _ = it["d"].cpu()
            else:
                ctx64.invert(it["mesh"], it["obs"], it["d_obs"], it["w"], lam=-1.0, tol=it["tol"],
                             max_iter=it["max_iter"], m_out=it["m_out"], prec=g.GRAV_FP64)
                _ = it["m_out"].cpu()
            lat_b.append(time.perf_counter() - t0 - it["t"])
            if progress:
                print(f"[serve] fp64 fifo {len(lat_b)}/{nb}", file=sys.stderr, flush=True)
        nd = len(lat_b)
        b50, b99 = _percentiles(lat_b)
        s50, s99 = _percentiles(lat[:nd])
        res["fp64_fifo_baseline"] = {"requests": nd, "p50_s": b50, "p99_s": b99,
                                     "wall_s": time.perf_counter() - t0,
                                     "batched_same_requests_p50_s": s50,
                                     "batched_same_requests_p99_s": s99}
        ctx64.close()
    ctx.close()
    return res


def run_serve(args) -> int:
    """The whole serving stream (--serve-requests of 200) through the server,
    and --serve-baseline-requests of it through the FP64 FIFO."""
    import torch
    import paper_2602_03857_amd as g
    dev = torch.device("cuda", 0)
    res = serve_replay(g, torch, dev, args.serve_requests, args.serve_max_active,
                       args.serve_budget_gb, args.serve_baseline_requests)
    print(json.dumps({"metric": "CG solve p50/p99 latency, serving stream", "serving": res}),
          flush=True)
    return 0


def run_cg_full(args) -> int:
    """The paper-scale inversion as configured: 178,797 observations over
    3,307,500 prisms, data = G m_true + 2 % relative Gaussian noise, depth
    weights w = (z + 25 m)^-1, lambda = 1e-2 trace(G C G^T) / N, exactly 50
    CG iterations on the data-space system, mixed precision.  The synthetic
    data are generated with the mixed forward itself (its 4e-7 error is far
    below the 2 % noise); this mode times the solve, it checks no parity."""
    import torch
    import paper_2602_03857_amd as g
    p = workloads.paper_scale()
    dev = torch.device("cuda", 0)
    mesh = g.DeviceMesh.from_mesh(p.mesh, dev)
    obs = g.DeviceObs.from_survey(p.obs, dev)
    m_true = torch.as_tensor(p.m, device=dev)
    w = torch.as_tensor(p.wdepth, device=dev)
    with g.Context(0, validate=True) as ctx:
        d = ctx.forward(mesh, obs, m_true, prec=g.GRAV_MIXED)
        draws = torch.as_tensor(p.noise_draws, device=dev)
        d_obs = d + p.noise_level * torch.sqrt(torch.mean(d * d)) * draws
        torch.cuda.synchronize()
        print("[cg] data ready; solving", file=sys.stderr, flush=True)
        ctx.set_timing(True)
        t0 = time.perf_counter()
        m, d_pred, info = ctx.invert(mesh, obs, d_obs, w, lam=-1.0, fixed_iters=p.cg_iters,
                                     want_pred=True, prec=g.GRAV_MIXED)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        tr_ms, _ = ctx.kernel_time("trace_mixed")
        f_ms, f_n = ctx.kernel_time("forward_mixed")
        a_ms, a_n = ctx.kernel_time("adjoint_mixed")
    misfit = float(torch.linalg.norm(d_pred - d_obs) / torch.linalg.norm(d_obs))
    noise = float(p.noise_level * torch.sqrt(torch.mean(d * d)) * torch.linalg.norm(draws)
                  / torch.linalg.norm(d_obs))
    # outside the iterations: the trace sweep, the final adjoint (m) and forward (d_pred)
    per_iter = (t - 1e-3 * (tr_ms + f_ms / max(f_n, 1) + a_ms / max(a_n, 1))) / p.cg_iters
    out = {"metric": "paper-scale data-space CG solve (178,797 obs x 3,307,500 prisms, 50 "
                     "iterations, GRAV_MIXED)",
           "solve_s": t, "iterations": info["iters"], "cg_iterations_per_s": 1.0 / per_iter,
           "trace_s": 1e-3 * tr_ms, "forward_kernel_ms_avg": f_ms / max(f_n, 1),
           "adjoint_kernel_ms_avg": a_ms / max(a_n, 1), "relres": info["relres"],
           "lambda": info["lambda_used"], "data_misfit_rel": misfit, "noise_rel": noise,
           "data": "synthetic (seeded paper-scale survey, model and noise)"}
    print(json.dumps(out), flush=True)
    return 0


def run_cg_compare(args) -> int:
    """Paper-scale solver evidence on the configured inversion (178,797 obs x
    3,307,500 prisms, 2 % noise, lambda = 1e-2 trace / N, plain CG from 0):
    (1) the relative-residual history of the first --cg-compare-iters
    iterations in GRAV_MIXED and in GRAV_FP64, entry by entry, and the two
    recovered densities after them; (2) plain against Jacobi-preconditioned
    CG (GRAV_MIXED) over --cg-jacobi-iters iterations: the iteration at which
    each first reaches a relative residual of 0.5, 0.3, 0.2 and 0.15."""
    import torch
    import paper_2602_03857_amd as g
    p = workloads.paper_scale()
    dev = torch.device("cuda", 0)
    mesh = g.DeviceMesh.from_mesh(p.mesh, dev)
    obs = g.DeviceObs.from_survey(p.obs, dev)
    m_true = torch.as_tensor(p.m, device=dev)
    w = torch.as_tensor(p.wdepth, device=dev)
    out = {"metric": "paper-scale CG: mixed vs FP64 residual histories; plain vs Jacobi",
           "data": "synthetic (seeded paper-scale survey, model and noise)"}
    with g.Context(0, validate=True) as ctx:
        d = ctx.forward(mesh, obs, m_true, prec=g.GRAV_MIXED)
        draws = torch.as_tensor(p.noise_draws, device=dev)
        d_obs = d + p.noise_level * torch.sqrt(torch.mean(d * d)) * draws
        torch.cuda.synchronize()
        k = args.cg_compare_iters
        hist, dens = {}, {}
        for prec, tag in ((g.GRAV_MIXED, "mixed"), (g.GRAV_FP64, "fp64")):
            t0 = time.perf_counter()
            m, _, info = ctx.invert(mesh, obs, d_obs, w, lam=-1.0, tol=0.0, max_iter=k,
                                    history_cap=k, prec=prec)
            torch.cuda.synchronize()
            hist[tag] = info["history"]
            dens[tag] = m.clone()
            out[f"{tag}_solve_s"] = time.perf_counter() - t0
            out[f"{tag}_lambda"] = info["lambda_used"]
            print(f"[cg-compare] {tag}: {k} iterations in {out[f'{tag}_solve_s']:.1f} s",
                  file=sys.stderr, flush=True)
        out["history_mixed"] = hist["mixed"]
        out["history_fp64"] = hist["fp64"]
        out["history_max_rel_diff"] = float(max(abs(a - b) / b for a, b in
                                                zip(hist["mixed"], hist["fp64"])))
        out["lambda_rel_diff"] = abs(out["mixed_lambda"] - out["fp64_lambda"]) / out["fp64_lambda"]
        out["density_rel_l2_mixed_vs_fp64"] = float(
            torch.linalg.norm(dens["mixed"] - dens["fp64"]) / torch.linalg.norm(dens["fp64"]))
        j = args.cg_jacobi_iters
        if j > 0:
            for pc, tag in ((0, "plain"), (1, "jacobi")):
                t0 = time.perf_counter()
                _, _, info = ctx.invert(mesh, obs, d_obs, w, lam=-1.0, tol=0.0, max_iter=j,
                                        history_cap=j, precond=pc, prec=g.GRAV_MIXED)
                torch.cuda.synchronize()
                h = info["history"]
                out[f"{tag}_history"] = h
                out[f"{tag}_solve_s"] = time.perf_counter() - t0
                out[f"{tag}_iters_to"] = {str(th): next((i + 1 for i, r in enumerate(h) if r <= th),
                                                        None) for th in (0.5, 0.3, 0.2, 0.15)}
                print(f"[cg-compare] {tag}: {j} iterations in {out[f'{tag}_solve_s']:.1f} s",
                      file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)
    return 0


def run_profile_op(args) -> int:
    """Only one operator at paper scale (178,797 obs x 3,307,500 prisms,
    GRAV_MIXED), args.steps times after args.warmup untimed calls: the target
    of the counter and kernel-trace runs of a single sweep ("multi": the
    split-bf16 multi-model forward of 64 models at 10,000 obs x 500,000
    prisms instead)."""
    import torch
    import paper_2602_03857_amd as g
    p = workloads.paper_scale()
    dev = torch.device("cuda", 0)
    mesh = g.DeviceMesh.from_mesh(p.mesh, dev)
    obs = g.DeviceObs.from_survey(p.obs, dev)
    m = torch.as_tensor(p.m, device=dev)
    v = torch.as_tensor(p.probe_v, device=dev)
    w = torch.as_tensor(p.wdepth, device=dev)
    out_n = torch.empty(p.obs.n, dtype=torch.float64, device=dev)
    out_m = torch.empty(p.mesh.ncells, dtype=torch.float64, device=dev)
    ops = {
        "forward": ("forward_mixed", lambda c: c.forward(mesh, obs, m, out_n, prec=g.GRAV_MIXED)),
        "adjoint": ("adjoint_mixed", lambda c: c.adjoint(mesh, obs, v, out_m, prec=g.GRAV_MIXED)),
        "dataspace": ("adjoint_mixed", lambda c: c.dataspace_apply(mesh, obs, w, 1e-12, v, out_n,
                                                                   prec=g.GRAV_MIXED)),
        "trace": ("trace_mixed", lambda c: c.trace(mesh, obs, w, prec=g.GRAV_MIXED)),
    }
    if args.profile_op == "multi":
        # 64 density models on the 100 x 100 x 50 mesh with 10,000 stations
        p3 = workloads.ellipsoids_100x100x50()
        mesh = g.DeviceMesh.from_mesh(p3.mesh, dev)
        obs = g.DeviceObs.from_survey(p3.obs, dev)
        models = torch.as_tensor(workloads.smoothed_box_models(p3.mesh).astype(np.float32),
                                 device=dev)
        D = torch.empty((p3.obs.n, models.shape[1]), dtype=torch.float32, device=dev)
        ops["multi"] = ("multi_bf16x3", lambda c: c.forward_multi(mesh, obs, models, D,
                                                                  prec=g.GRAV_MIXED_BF16X3))
    kname, call = ops[args.profile_op]
    with g.Context(0, validate=False) as ctx:
        ctx.set_timing(True)
        for _ in range(args.warmup):
            call(ctx)
        torch.cuda.synchronize()
        ctx.reset_timing()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            call(ctx)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        k_ms, k_n = ctx.kernel_time(kname)
    print(json.dumps({"profile_op": args.profile_op, "steps": args.steps,
                      "ms_per_call": 1e3 * dt / max(args.steps, 1), "kernel": kname,
                      "kernel_ms_avg": k_ms / max(k_n, 1), "launches": k_n}), flush=True)
    return 0


def run_cg_graph(args) -> int:
    """Small CG solves with the kernels launched one by one against the same
    iterations replayed from a HIP graph (grav_cg_opts.graph)."""
    import torch
    import paper_2602_03857_amd as g
    from oracle import prism
    dev = torch.device("cuda", 0)
    res = {}
    for p in (workloads.dykes_32x32x16(), workloads.random_case(7, 60, 50, 40, 5000)):
        mesh = g.DeviceMesh.from_mesh(p.mesh, dev)
        obs = g.DeviceObs.from_survey(p.obs, dev)
        d = torch.as_tensor(prism.forward(p.mesh, p.obs, p.m), device=dev)
        w = torch.as_tensor(p.wdepth, device=dev)
        row = {"n_obs": p.obs.n, "n_cells": p.mesh.ncells}
        with g.Context(0, validate=False) as ctx:
            for graph in (False, True):
                ctx.invert(mesh, obs, d, w, lam=-1.0, tol=1e-6, max_iter=300, graph=graph)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    _, _, info = ctx.invert(mesh, obs, d, w, lam=-1.0, tol=1e-6, max_iter=300,
                                            graph=graph)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t0) / args.steps
                key = "graph" if graph else "eager"
                row[key + "_ms_per_solve"] = ms
                row[key + "_iterations"] = info["iters"]
        row["speedup"] = row["eager_ms_per_solve"] / row["graph_ms_per_solve"]
        res[p.name] = row
    print(json.dumps({"metric": "CG solve time, kernels one by one vs graph replay", "solves": res}),
          flush=True)
    return 0


def run_issue_probe(args) -> int:
    """Measure the issue rates behind the roofline's slot weights."""
    import torch  # noqa: F401
    import paper_2602_03857_amd as g
    with g.Context(0) as ctx:
        r = ctx.issue_rates()
        pr = ctx.issue_pair_rates()
    fma = r["fma32"]
    # half FMA, half another class: the rate of the two halves run in sequence
    serial = {"log": 2.0 / (1.0 / fma + 1.0 / r["log"]),
              "select": 2.0 / (1.0 / fma + 1.0 / pr["select"])}
    pairs = {k: {"rate": pr[k], "over_sequential": pr[k] / serial["log" if "log" in k else "select"]}
             for k in pr if k != "select"}
    out = {"metric": "gfx950 issue rates (chain steps/s summed over lanes)", "rates": r,
           "select_alone": pr["select"], "pairs": pairs,
           "fma32_per_peak_slot": fma / PEAK_SLOTS,
           "slots_per_instruction": {k: (fma / r[k] - fma / r["add32"] if k in ("log", "rcp", "sqrt")
                                         else fma / r[k]) for k in r},
           "weights_used": {"transcendental": TRANS_COST, "fp64": FP64_COST}}
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-model timing")
    ap.add_argument("--cg-iters", type=int, default=3, help="CG iterations timed for it/s")
    ap.add_argument("--serve", action="store_true", help="replay the serving stream instead")
    ap.add_argument("--cg-full", action="store_true",
                    help="time the paper-scale 50-iteration CG solve instead")
    ap.add_argument("--cg-graph", action="store_true",
                    help="small CG solves: kernels one by one vs iterations replayed from a HIP graph")
    ap.add_argument("--cg-compare", action="store_true",
                    help="paper-scale CG: mixed vs FP64 histories, plain vs Jacobi")
    ap.add_argument("--cg-compare-iters", type=int, default=6)
    ap.add_argument("--cg-jacobi-iters", type=int, default=50)
    ap.add_argument("--issue-probe", action="store_true",
                    help="measure the instruction issue rates behind the roofline weights")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter calibration)")
    ap.add_argument("--profile-op", choices=("forward", "adjoint", "dataspace", "multi", "trace"),
                    help="only time this operator at paper scale (profiling runs)")
    ap.add_argument("--serve-extras-requests", type=int, default=60,
                    help="requests of the serving stream replayed in the default run (0 = none)")
    ap.add_argument("--serve-extras-fifo", type=int, default=10,
                    help="of those, requests replayed through the FP64 FIFO (at most 30 s)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-baseline-requests", type=int, default=40)
    ap.add_argument("--serve-max-active", type=int, default=64)
    ap.add_argument("--serve-budget-gb", type=int, default=48)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: --gpus {args.gpus} is not supported "
              "(the library is single-device; multi-GPU sharding is a design note only).",
              file=sys.stderr)
        return 2

    if args.serve:
        return run_serve(args)
    if args.cg_full:
        return run_cg_full(args)
    if args.cg_compare:
        return run_cg_compare(args)
    if args.issue_probe:
        return run_issue_probe(args)
    if args.cg_graph:
        return run_cg_graph(args)
    if args.profile_op:
        return run_profile_op(args)
    if args.copy_probe:
        import torch
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "launches": 3}), flush=True)
        return 0

    p = workloads.paper_scale()
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
        # by path: importing the package would try to load the missing library
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "grav_build", os.path.join(ROOT, "paper_2602_03857_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
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

    ncols = (p.mesh.nx + 1) * (p.mesh.ny + 1)
    kdeep = first_deep_layer(p.mesh.zn)
    nz = p.mesh.nz
    segs = ncols * nz
    costs = sweep_costs(n, ncols, nz, kdeep)
    instr, slots_fwd = costs["fwd"]
    k_s = k_avg_ms * 1e-3
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("source_hash") == kernel_source_hash():
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "alu", "achieved": slots_fwd / k_s / 1e12, "peak": PEAK_SLOTS / 1e12,
                "unit": "T lane-slots/s", "frac": slots_fwd / k_s / PEAK_SLOTS, "traffic": traffic,
                "kernel": "k_forward_mixed", "kernel_ms": k_avg_ms,
                "segments_per_launch": segs * n, "slots_per_launch": slots_fwd,
                "frac_unweighted_instructions": instr / k_s / PEAK_SLOTS}

    # error vs the oracle on the stored rows
    extras = {}
    gold_path = os.path.join(ROOT, "tests", "golden", "paper_scale_rows.npz")
    if os.path.exists(gold_path):
        gold = np.load(gold_path)
        dn = d.cpu().numpy()[gold["rows"]]
        extras["rel_l2_vs_fp64_oracle_2000_rows"] = float(
            np.linalg.norm(dn - gold["d"]) / np.linalg.norm(gold["d"]))

    if not args.no_extras:
        v = torch.as_tensor(p.probe_v, device=dev)
        gt = torch.empty(M, dtype=torch.float64, device=dev)
        ctx.adjoint(mesh, obs, v, gt, prec=g.GRAV_MIXED)
        torch.cuda.synchronize()
        ctx.reset_timing()
        t0 = time.perf_counter()
        ctx.adjoint(mesh, obs, v, gt, prec=g.GRAV_MIXED)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        a_ms, a_n = ctx.kernel_time("adjoint_mixed")
        extras["adjoint_pairs_per_s"] = pairs / t_adj
        extras["adjoint_ms"] = 1e3 * t_adj
        extras["adjoint_kernel_ms"] = a_ms / max(a_n, 1)
        # the same edge segments at the adjoint's own instruction counts,
        # against the same peak
        extras["adjoint_roofline_frac"] = (costs["adj"][1] / (extras["adjoint_kernel_ms"] * 1e-3)
                                           / PEAK_SLOTS)

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
            extras["cg_timed_iterations"] = args.cg_iters
            extras["cg_total_s"] = t_cg
            extras["cg_relres"] = info["relres"]

    if not args.no_extras and not args.no_multi:
        extras.update(multi_model_extras(g, torch, dev))
    if not args.no_extras:
        extras.update(ellipsoids_extras(g, torch, dev))
    if not args.no_extras and args.serve_extras_requests > 0:
        # the metric's second half: CG solve latency under the serving stream
        extras["serving"] = serve_replay(g, torch, dev, args.serve_extras_requests,
                                         args.serve_max_active, args.serve_budget_gb,
                                         args.serve_extras_fifo, fifo_budget_s=30.0)

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
        "data": "synthetic (seeded paper-scale survey and model)",
        "config": {"workload": "paper_scale: G m, 178,797 obs x 3,307,500 prisms (150x150x147, "
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
