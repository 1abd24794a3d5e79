"""GPU parity: the HIP operators (called through the C ABI) against the FP64
CPU oracle on the same seeded inputs.

Tolerances: GRAV_FP64 to 1e-10 relative L2 (both are FP64; only summation
order differs), except the plain FP64 adjoint on the full-size meshes, whose
cap follows the rounding scale of its corner-term sums (_f64_corner_cap);
GRAV_MIXED to 1e-5 relative L2 for gz (the accuracy target of the mixed path)
and 1e-4 relative L2 for the recovered density."""
import os

import numpy as np
import pytest

from oracle import trend as trend_oracle
from oracle import prism, inversion, GAMMA
import workloads
from tests._util import load_package, rel_l2, to_np

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-10
TOL_MIXED = 1e-5
EPS32 = 2.0 ** -24
# Each FP32 edge term is accurate to a few units of its own magnitude, so an
# edge-wise sum is accurate to C_TERMS * eps32 * (sum of |terms|).
C_TERMS = 16.0
HERE = os.path.dirname(os.path.abspath(__file__))


# The plain FP64 adjoint sums corner terms Psi(node - obs) of magnitude about
# R ln R (Eq. 2) over the observations and then takes the 8-term vertex
# alternation of Eq. 1, which cancels all but about (a/R)^3 / ln R of them for
# a cell of size a at distance R.  Its rounding scale is therefore
# eps64 * sum |corner terms|, not eps64 * |value|: at 100 x 100 x 50 cells (R/a
# up to about 150) about 1e-9 of the value, at paper scale about 1e-8.  Its
# relative L2 cap is the L2 form of the same C_TERMS * eps64 * sum |terms|
# bound the entrywise check applies, never below TOL_F64.


def _f64_corner_cap(ref, scale):
    return max(TOL_F64, C_TERMS * 2.0 ** -53 * float(np.linalg.norm(scale) / np.linalg.norm(ref)))


def _check_termwise(name, got, ref, scale, eps=EPS32, informative=True, rel_cap=TOL_MIXED):
    """|got - ref| <= C_TERMS * eps * scale elementwise (scale = sum of the
    magnitudes of the terms the GPU adds up, from the oracle).

    informative: the probe is sign-definite, so every entry is a sum without
    cancellation between observations; then the bound must also lie below
    |ref| at every checked entry (an all-zero output fails it) and the
    relative L2 error must meet rel_cap."""
    bound = C_TERMS * eps * scale
    ratio = np.abs(got - ref) / bound
    err = rel_l2(got, ref)
    print(f"[parity] {name}: rel L2 = {err:.3e} (cap {rel_cap:.1e}), worst err / term bound = "
          f"{ratio.max():.3f}, largest bound / |value| = {np.max(bound / np.abs(ref)):.2e}",
          flush=True)
    assert np.all(ratio <= 1.0)
    if informative:
        assert np.all(bound < np.abs(ref)), "term bound does not exclude a zero output"
        assert err <= rel_cap


@pytest.fixture(scope="module")
def g():
    pkg = load_package()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return pkg


@pytest.fixture(scope="module")
def ctx(g):
    c = g.Context(device=0)
    yield c
    c.close()


def _dev(g, p):
    return g.DeviceMesh.from_mesh(p.mesh), g.DeviceObs.from_survey(p.obs)


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _report(name, err):
    print(f"[parity] {name}: rel L2 = {err:.3e}", flush=True)


# ------------------------------------------------------------------ forward

@pytest.mark.parametrize("prec_name", ["GRAV_FP64", "GRAV_MIXED"])
@pytest.mark.parametrize("case", [
    dict(seed=1, nx=13, ny=11, nz=7, n=333, on_nodes=20, on_top=40),
    dict(seed=2, nx=5, ny=3, nz=2, n=1, on_nodes=0, on_top=0),
    dict(seed=3, nx=1, ny=1, nz=1, n=65, on_nodes=10, on_top=10),
    dict(seed=4, nx=40, ny=9, nz=33, n=257, on_nodes=30, on_top=30),
])
def test_forward_random_ragged(g, ctx, prec_name, case):
    p = workloads.random_case(case["seed"], case["nx"], case["ny"], case["nz"], case["n"],
                              on_nodes=case["on_nodes"], on_top=case["on_top"])
    mesh, obs = _dev(g, p)
    d = to_np(ctx.forward(mesh, obs, _t(p.m), prec=getattr(g, prec_name)))
    ref = prism.forward(p.mesh, p.obs, p.m)
    err = rel_l2(d, ref)
    _report(f"forward {prec_name} {case}", err)
    assert err <= (TOL_F64 if prec_name == "GRAV_FP64" else TOL_MIXED)
    assert np.all(np.isfinite(d))


@pytest.mark.parametrize("prec_name", ["GRAV_FP64", "GRAV_MIXED"])
def test_forward_dykes_32x32x16(g, ctx, prec_name):
    p = workloads.dykes_32x32x16()
    mesh, obs = _dev(g, p)
    d = to_np(ctx.forward(mesh, obs, _t(p.m), prec=getattr(g, prec_name)))
    ref = prism.forward(p.mesh, p.obs, p.m)
    err = rel_l2(d, ref)
    _report(f"forward dykes_32x32x16 {prec_name}", err)
    assert err <= (TOL_F64 if prec_name == "GRAV_FP64" else TOL_MIXED)
    assert np.max(np.abs(d - ref)) <= 10 * (TOL_F64 if prec_name == "GRAV_FP64" else TOL_MIXED) * np.max(np.abs(ref))


def _single_prism_positions():
    """Observation points around one prism: on its corners, edges and top
    face, and on shells at R/a = 0.5 ... 30 (all on or above the top)."""
    xs, ys, top = (0.0, 100.0), (0.0, 60.0), 20.0
    pts = []
    for x in (-50.0, 0.0, 37.0, 100.0, 160.0):
        for y in (-30.0, 0.0, 22.0, 60.0, 95.0):
            for h in (0.0, 1.0, 30.0):
                pts.append((x, y, top - h))
    rng = np.random.default_rng(42)
    c = np.array([50.0, 30.0, 55.0])
    for ratio in (0.5, 1.0, 3.0, 10.0, 30.0):
        for _ in range(40):
            d = rng.standard_normal(3)
            d[2] = -abs(d[2])
            d /= np.linalg.norm(d)
            o = c + ratio * 100.0 * d
            o[2] = min(o[2], top)
            pts.append(tuple(o))
    pts = np.array(pts)
    mesh = workloads.Mesh(np.array(xs), np.array(ys), np.array([top, 90.0]))
    return mesh, workloads.Survey(pts[:, 0], pts[:, 1], pts[:, 2])


@pytest.mark.parametrize("prec_name", ["GRAV_FP64", "GRAV_MIXED"])
def test_single_prism_singular_and_far_positions(g, ctx, prec_name):
    """Per point, one prism (100 x 60 x 70 m).  Bounds from the cancellation
    of each evaluation: FP64 sums 8 corner terms of size ~R ln R to a result
    ~V/R^2, so ~ eps64 R^3 ln R / V; the FP32 edge form sums 4 edge terms of
    size ~h to ~a_x a_y h z_c / R^3, so ~ eps32 R^3 / (a_x a_y z_c), z_c = the
    prism-centre depth below the point."""
    mesh_h, obs_h = _single_prism_positions()
    mesh, obs = g.DeviceMesh.from_mesh(mesh_h), g.DeviceObs.from_survey(obs_h)
    m = np.array([1000.0])
    d = to_np(ctx.forward(mesh, obs, _t(m), prec=getattr(g, prec_name)))
    ref = prism.forward_literal(mesh_h, obs_h, m)
    R = np.sqrt((obs_h.x - 50.0) ** 2 + (obs_h.y - 30.0) ** 2 + (obs_h.z - 55.0) ** 2)
    R = np.maximum(R, 100.0)
    zc = 55.0 - obs_h.z
    rel = np.abs(d - ref) / np.abs(ref)
    if prec_name == "GRAV_FP64":
        bound = np.maximum(1e-12, 200 * 2.0 ** -53 * R ** 3 * np.log(R) / (100 * 60 * 70))
    else:
        bound = np.maximum(2e-6, 100 * EPS32 * R ** 3 / (100 * 60 * zc))
    worst = int(np.argmax(rel / bound))
    near = R <= 300.0
    print(f"[parity] single prism {prec_name}: worst rel/bound {rel[worst] / bound[worst]:.2f} "
          f"(rel {rel[worst]:.2e}); near field (R <= 3a) max rel {rel[near].max():.2e}", flush=True)
    assert np.all(np.isfinite(d))
    assert np.all(rel <= bound)
    assert rel[near].max() <= (1e-12 if prec_name == "GRAV_FP64" else 1e-4)


# ------------------------------------------------------------------ adjoint

@pytest.mark.parametrize("prec_name", ["GRAV_FP64", "GRAV_MIXED"])
@pytest.mark.parametrize("case", [
    dict(seed=5, nx=13, ny=11, nz=7, n=333, on_nodes=20, on_top=40),
    dict(seed=6, nx=31, ny=17, nz=19, n=70, on_nodes=5, on_top=5),
    dict(seed=7, nx=2, ny=3, nz=1, n=1, on_nodes=1, on_top=1),
    # 40 layers, first deep layer 12: the 12 layers above it in one chunk on
    # the general path, the deep ones in two chunks of 14 (layers 12-25 and
    # 26-39), each walk carrying its angle over 14 layers
    dict(seed=13, nx=9, ny=8, nz=40, n=61, on_nodes=5, on_top=5),
])
def test_adjoint_random_ragged(g, ctx, prec_name, case):
    """Two probes: v = |N(0, 1)| (sign-definite: every entry of G^T v is a sum
    without cancellation, checked to the operator tolerance) and v = N(0, 1)
    (entries that cancel across observations, checked against the rounding
    scale of the terms they add)."""
    p = workloads.random_case(case["seed"], case["nx"], case["ny"], case["nz"], case["n"],
                              on_nodes=case["on_nodes"], on_top=case["on_top"])
    mesh, obs = _dev(g, p)
    prec = getattr(g, prec_name)
    cells = np.arange(p.mesh.ncells)
    for probe, signed in ((np.abs(p.probe_v), False), (p.probe_v, True)):
        gt = to_np(ctx.adjoint(mesh, obs, _t(probe), prec=prec))
        ref = prism.adjoint(p.mesh, p.obs, probe)
        label = f"adjoint {prec_name} {'signed' if signed else '|v|'} {case}"
        if prec_name == "GRAV_FP64":
            err = rel_l2(gt, ref)
            _report(label, err)
            assert err <= TOL_F64
        else:
            scale = prism.adjoint_abs_scale(p.mesh, p.obs, probe, cells)
            _check_termwise(label, gt, ref, scale, informative=not signed)


def _first_deep_layer(zn, ratio=9.0, min_depth=1e-3):
    """First layer from which every layer's top lies at least `ratio`
    thicknesses and `min_depth` below the mesh top."""
    k = len(zn) - 1
    while k > 0 and zn[k - 1] - zn[0] >= ratio * (zn[k] - zn[k - 1]) and zn[k - 1] - zn[0] >= min_depth:
        k -= 1
    return k


@pytest.mark.parametrize("prec_name", ["GRAV_FP64", "GRAV_MIXED"])
def test_adjoint_graded_layers_two_general_chunks(g, ctx, prec_name):
    """Layers 3 m thick, one of 8 m at index 16, then 4 m: the first deep
    layer is 17, so the mixed adjoint chunks the 17 layers above it in two
    (9 and 8 layers) and the 33 deep ones in three walks of 11 (odd length),
    which fill all ceil(50 / 16) + 1 chunk indices of the launch."""
    p = workloads.random_case(21, 8, 7, 1, 61, on_nodes=5, on_top=5)
    hz = np.array([3.0] * 16 + [8.0] + [4.0] * 33)
    zn = np.concatenate([[0.0], np.cumsum(hz)])
    assert _first_deep_layer(zn) == 17
    m = workloads.Mesh(p.mesh.xn, p.mesh.yn, zn)
    mesh = g.DeviceMesh.from_mesh(m)
    obs = g.DeviceObs.from_survey(p.obs)
    prec = getattr(g, prec_name)
    cells = np.arange(m.ncells)
    for probe, signed in ((np.abs(p.probe_v), False), (p.probe_v, True)):
        gt = to_np(ctx.adjoint(mesh, obs, _t(probe), prec=prec))
        ref = prism.adjoint(m, p.obs, probe)
        label = f"adjoint graded {prec_name} {'signed' if signed else '|v|'}"
        if prec_name == "GRAV_FP64":
            err = rel_l2(gt, ref)
            _report(label, err)
            assert err <= TOL_F64
        else:
            scale = prism.adjoint_abs_scale(m, p.obs, probe, cells)
            _check_termwise(label, gt, ref, scale, informative=not signed)


@pytest.mark.parametrize("prec_name", ["GRAV_FP64", "GRAV_MIXED"])
def test_adjoint_dot_product(g, ctx, prec_name):
    """<G m, v> = <m, G^T v> on the GPU operators themselves."""
    p = workloads.random_case(8, 24, 20, 12, 500, on_top=50)
    mesh, obs = _dev(g, p)
    prec = getattr(g, prec_name)
    d = to_np(ctx.forward(mesh, obs, _t(p.m), prec=prec))
    gt = to_np(ctx.adjoint(mesh, obs, _t(p.probe_v), prec=prec))
    lhs, rhs = np.dot(d, p.probe_v), np.dot(p.m, gt)
    scale = np.linalg.norm(d) * np.linalg.norm(p.probe_v)
    assert abs(lhs - rhs) <= (1e-12 if prec_name == "GRAV_FP64" else 1e-6) * scale


# ------------------------------------------------------------------ data space / trace

@pytest.mark.parametrize("prec_name", ["GRAV_FP64", "GRAV_MIXED"])
@pytest.mark.parametrize("case", [
    (9, 12, 10, 8, 150),
    # 40 layers, first deep layer 12: the adjoint's layer chunks start at 0
    # (general path), 12 and 26 (deep-layer path)
    (13, 9, 8, 40, 61),
])
def test_dataspace_apply_matches_oracle(g, ctx, prec_name, case):
    p = workloads.random_case(*case, on_top=20, model="blocky")
    mesh, obs = _dev(g, p)
    lam = 3.7e-14
    for probe, label in ((p.probe_v, "signed"), (np.abs(p.probe_v), "|v|")):
        out = to_np(ctx.dataspace_apply(mesh, obs, _t(p.wdepth), lam, _t(probe),
                                        prec=getattr(g, prec_name)))
        ref = inversion.dataspace_apply(p.mesh, p.obs, p.wdepth, lam, probe)
        err = rel_l2(out, ref)
        _report(f"dataspace {prec_name} {label} {case}", err)
        assert err <= (TOL_F64 if prec_name == "GRAV_FP64" else TOL_MIXED)


@pytest.mark.parametrize("prec_name", ["GRAV_FP64", "GRAV_MIXED"])
@pytest.mark.parametrize("case", [
    (10, 9, 14, 6, 129),
    (11, 6, 7, 24, 97),    # first deep layer 10 of 24: both edge formulas
])
def test_trace_and_diagonal(g, ctx, prec_name, case):
    import torch
    p = workloads.random_case(*case, on_top=10, on_nodes=10)
    mesh, obs = _dev(g, p)
    cov = inversion.covariance_from_weights(p.wdepth)
    ref_diag = prism.weighted_row_sumsq(p.mesh, p.obs, cov)
    diag = torch.empty(p.obs.n, dtype=torch.float64, device="cuda")
    tr = ctx.trace(mesh, obs, _t(p.wdepth), diag=diag, prec=getattr(g, prec_name))
    tol = 1e-10 if prec_name == "GRAV_FP64" else 1e-5
    assert rel_l2(to_np(diag), ref_diag) <= tol
    assert abs(tr - ref_diag.sum()) <= tol * ref_diag.sum()


# ------------------------------------------------------------------ inversion

def _dykes_reference():
    p = workloads.dykes_32x32x16()
    G = np.stack([prism.sensitivity_row(p.mesh, p.obs.x[o], p.obs.y[o], p.obs.z[o])
                  for o in range(p.obs.n)])
    cov = inversion.covariance_from_weights(p.wdepth)
    d_clean = G @ p.m
    d_obs = inversion.add_noise(d_clean, p.noise_draws, p.noise_level)
    trace = float(np.einsum("ok,k,ok->", G, cov, G))
    lam = inversion.lambda_rule(trace, p.obs.n)
    m_chol, _ = inversion.invert_dense(G, cov, lam, d_obs)
    return p, G, d_obs, trace, lam, m_chol


@pytest.fixture(scope="module")
def dykes_ref():
    return _dykes_reference()


@pytest.mark.parametrize("prec_name", ["GRAV_FP64", "GRAV_MIXED"])
def test_invert_dykes_32x32x16_vs_cholesky(g, ctx, dykes_ref, prec_name):
    p, G, d_obs, trace, lam, m_chol = dykes_ref
    mesh, obs = _dev(g, p)
    m, d_pred, info = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=-1.0, tol=p.cg_tol,
                                 max_iter=2000, want_pred=True, prec=getattr(g, prec_name))
    print(f"[parity] invert dykes_32x32x16 {prec_name}: {info}", flush=True)
    assert info["converged"] and info["relres"] <= p.cg_tol
    assert abs(info["trace"] - trace) <= 1e-5 * trace
    err = rel_l2(to_np(m), m_chol)
    _report(f"invert dykes_32x32x16 {prec_name} density", err)
    assert err <= 1e-4
    assert rel_l2(to_np(d_pred), G @ m_chol) <= 1e-4


@pytest.mark.parametrize("prec_name", ["GRAV_FP64", "GRAV_MIXED"])
def test_invert_jacobi_preconditioned(g, ctx, dykes_ref, prec_name):
    """Jacobi-preconditioned CG (M = diag(G C G^T) + lambda I) reaches the same
    unique solution of Eq. 11 as the Cholesky solve."""
    p, G, d_obs, trace, lam, m_chol = dykes_ref
    mesh, obs = _dev(g, p)
    prec = getattr(g, prec_name)
    _, _, plain = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=-1.0, tol=p.cg_tol,
                             max_iter=2000, prec=prec)
    m, _, info = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=-1.0, tol=p.cg_tol,
                            max_iter=2000, prec=prec, precond=1)
    print(f"[parity] invert dykes_32x32x16 {prec_name} Jacobi: {info['iters']} iterations "
          f"(plain CG {plain['iters']})", flush=True)
    assert info["converged"] and info["relres"] <= p.cg_tol
    err = rel_l2(to_np(m), m_chol)
    _report(f"invert dykes_32x32x16 {prec_name} Jacobi density", err)
    assert err <= 1e-4


# CG in floating point: the recursive residual of this system (kappa ~ 2e3)
# follows the exact-arithmetic sequence for about ten iterations; after that a
# relative perturbation of the operator as small as 1e-15 changes it by per
# cent (the oracle shows this on the dense system), so iteration counts and
# late residuals are compared with a margin, early ones tightly.
_EARLY = 8


def test_invert_misfit_history_plain_cg(g, ctx, dykes_ref):
    """Misfit log of plain CG against the oracle's residual history."""
    p, G, d_obs, trace, lam, m_chol = dykes_ref
    mesh, obs = _dev(g, p)
    cov = inversion.covariance_from_weights(p.wdepth)
    A = inversion.dataspace_matrix(G, cov, lam)
    _, it_ref, hist = inversion.conjugate_gradient(lambda v: A @ v, d_obs, tol=1e-6, max_iter=500)
    _, _, info = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, tol=1e-6, max_iter=500,
                            prec=g.GRAV_FP64, history_cap=30)
    assert len(info["history"]) == 30 < info["iters"]
    assert abs(info["iters"] - it_ref) <= max(3, it_ref // 10)
    np.testing.assert_allclose(info["history"][:_EARLY], hist[1:1 + _EARLY], rtol=1e-6)
    _, _, full = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, tol=1e-6, max_iter=500,
                            prec=g.GRAV_FP64, history_cap=1000)
    h = full["history"]
    assert len(h) == full["iters"] and h[-1] == full["relres"] <= 1e-6 < min(h[:-1])


def test_invert_warm_start_and_resume(g, ctx, dykes_ref):
    """Warm start / resume: CG from an oracle iterate (10 oracle iterations)
    follows the oracle's resumed history and returns its final iterate in
    y_out; from the Cholesky solution no iteration is needed; the restarted
    policy resumes the same way."""
    import torch
    p, G, d_obs, trace, lam, m_chol = dykes_ref
    mesh, obs = _dev(g, p)
    cov = inversion.covariance_from_weights(p.wdepth)
    A = inversion.dataspace_matrix(G, cov, lam)
    y10, _, _ = inversion.conjugate_gradient(lambda v: A @ v, d_obs, fixed_iters=10)
    _, it_ref, hist_ref = inversion.conjugate_gradient(lambda v: A @ v, d_obs, tol=1e-6,
                                                       max_iter=500, y0=y10)
    y_out = torch.empty(p.obs.n, dtype=torch.float64, device="cuda")
    m, _, info = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, tol=1e-6, max_iter=500,
                            prec=g.GRAV_FP64, y0=_t(y10), y_out=y_out, history_cap=1000)
    print(f"[parity] resumed CG: {info['iters']} iterations (oracle {it_ref})", flush=True)
    assert info["converged"] and abs(info["iters"] - it_ref) <= max(3, it_ref // 10)
    np.testing.assert_allclose(info["history"][:_EARLY], hist_ref[1:1 + _EARLY], rtol=1e-6)
    yo = to_np(y_out)
    assert np.linalg.norm(d_obs - A @ yo) <= 2e-6 * np.linalg.norm(d_obs)
    assert rel_l2(to_np(m), cov * (G.T @ yo)) <= 1e-9
    y_ch = np.linalg.solve(A, d_obs)
    m2, _, info2 = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, tol=1e-6,
                              prec=g.GRAV_FP64, y0=_t(y_ch))
    assert info2["iters"] == 0 and info2["converged"] and rel_l2(to_np(m2), m_chol) <= 1e-8
    y_r, _, cyc, _ = inversion.restarted_cg(lambda v: A @ v, d_obs, 20, 30, 1e-6, y0=y10)
    m3, _, info3 = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, tol=1e-6, restart=20,
                              max_cycles=30, prec=g.GRAV_FP64, y0=_t(y10))
    assert info3["converged"] and abs(info3["cycles"] - cyc) <= 1
    assert rel_l2(to_np(m3), cov * (G.T @ y_r)) <= 2e-5


def test_invert_fixed_iterations_and_noconv(g, ctx, dykes_ref):
    p, G, d_obs, trace, lam, m_chol = dykes_ref
    mesh, obs = _dev(g, p)
    m, _, info = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, fixed_iters=5)
    assert info["iters"] == 5 and info["converged"]
    cov = inversion.covariance_from_weights(p.wdepth)
    A = inversion.dataspace_matrix(G, cov, lam)
    y, _, hist = inversion.conjugate_gradient(lambda v: A @ v, d_obs, fixed_iters=5)
    m_ref5 = cov * (G.T @ y)
    assert rel_l2(to_np(m), m_ref5) <= 1e-4
    assert abs(info["relres"] - hist[-1]) <= 1e-3 * hist[-1]
    m2, _, info2 = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, tol=1e-12, max_iter=3)
    assert not info2["converged"] and info2["iters"] == 3
    assert np.all(np.isfinite(to_np(m2)))


@pytest.mark.parametrize("prec_name,tol", [("GRAV_FP64", 1e-4), ("GRAV_FP64", 1e-6),
                                           ("GRAV_MIXED", 1e-4)])
def test_invert_restarted_policy(g, ctx, dykes_ref, prec_name, tol):
    """Restarted CG (Section 2.2 policy: at most 20 inner iterations in at most
    30 cycles, step backtracking) against the oracle's restarted CG on the
    dense system of Eq. 11."""
    p, G, d_obs, trace, lam, m_chol = dykes_ref
    mesh, obs = _dev(g, p)
    cov = inversion.covariance_from_weights(p.wdepth)
    A = inversion.dataspace_matrix(G, cov, lam)
    log = []
    y_ref, iters_ref, cycles_ref, hist = inversion.restarted_cg(lambda v: A @ v, d_obs, 20, 30, tol,
                                                                log=log)
    m_ref = cov * (G.T @ y_ref)
    m, _, info = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, tol=tol, restart=20,
                            max_cycles=30, max_halvings=5, prec=getattr(g, prec_name),
                            history_cap=1000)
    print(f"[parity] restarted CG {prec_name} tol {tol}: iters {info['iters']} cycles "
          f"{info['cycles']} halvings {info['halvings']} relres {info['relres']:.3e} "
          f"(oracle {iters_ref} iterations, {cycles_ref} cycles)", flush=True)
    assert info["converged"] and info["relres"] <= tol
    assert abs(info["cycles"] - cycles_ref) <= 1
    # the mixed operator (relative error ~4e-7) perturbs the recursion sooner
    margin = iters_ref // 10 if prec_name == "GRAV_FP64" else iters_ref // 4
    assert abs(info["iters"] - iters_ref) <= max(3, margin)
    # misfit log: one entry per inner iteration; the early ones are the oracle's
    hlog = info["history"]
    assert len(hlog) == info["iters"]
    # (the mixed operator's ~4e-7 error moves the recursion off the exact
    # sequence after about five iterations)
    n_early, early = (_EARLY, 1e-6) if prec_name == "GRAV_FP64" else (4, 1e-3)
    np.testing.assert_allclose(hlog[:n_early], log[:n_early], rtol=early)
    err = rel_l2(to_np(m), m_ref)
    _report(f"restarted CG dykes_32x32x16 {prec_name} tol {tol} vs oracle", err)
    assert rel_l2(to_np(m), m_chol) <= 10 * tol and err <= 20 * tol


def test_invert_restarted_cycle_cap_and_errors(g, ctx, dykes_ref):
    p, G, d_obs, trace, lam, m_chol = dykes_ref
    mesh, obs = _dev(g, p)
    cov = inversion.covariance_from_weights(p.wdepth)
    A = inversion.dataspace_matrix(G, cov, lam)
    y_ref, _, _, hist = inversion.restarted_cg(lambda v: A @ v, d_obs, 5, 3, 1e-12)
    m, _, info = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, tol=1e-12, restart=5,
                            max_cycles=3, prec=g.GRAV_FP64)
    assert not info["converged"] and info["cycles"] == 3 and info["iters"] == 15
    # the FP64 node-sum operator differs from the dense literal G by ~1e-11
    # relative (eps64 (R/a)^3 ln R per prism); through 15 CG steps on this
    # system that moves the iterate by ~1e-5 (a 1e-14 perturbation moves it
    # 3e-7 in the oracle's own experiment)
    assert rel_l2(to_np(m), cov * (G.T @ y_ref)) <= 1e-4
    assert abs(info["relres"] - hist[-1]) <= 1e-3 * hist[-1]
    for bad in (dict(restart=5, max_cycles=0), dict(restart=5, precond=1),
                dict(restart=5, fixed_iters=3), dict(restart=-1), dict(restart=5, max_halvings=-1)):
        with pytest.raises(g.GravError):
            ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, tol=1e-4, **bad)


def test_invert_with_reference_model(g, ctx):
    p = workloads.random_case(11, 6, 5, 4, 40, model="blocky")
    G = np.stack([prism.sensitivity_row(p.mesh, p.obs.x[o], p.obs.y[o], p.obs.z[o])
                  for o in range(p.obs.n)])
    cov = inversion.covariance_from_weights(p.wdepth)
    d_obs = inversion.add_noise(G @ p.m, p.noise_draws, 0.01)
    m_ref = np.full(p.mesh.ncells, 0.1)
    lam = 1e-2 * float(np.einsum("ok,k,ok->", G, cov, G)) / p.obs.n
    m_chol, _ = inversion.invert_dense(G, cov, lam, d_obs, m_ref)
    mesh, obs = _dev(g, p)
    m, _, info = ctx.invert(mesh, obs, _t(d_obs), _t(p.wdepth), lam=lam, m_ref=_t(m_ref),
                            tol=1e-10, max_iter=500, prec=g.GRAV_FP64)
    assert rel_l2(to_np(m), m_chol) <= 1e-6


# ------------------------------------------------------------------ full-size workloads

def test_ellipsoids_100x100x50_forward_adjoint_sampled(g, ctx):
    """10,000 observations x 500,000 prisms: G m on 256 stored rows, G^T v
    (v = |probe|) on 64 stored cells, trace(G C G^T) and its diagonal at every
    observation, and the data-space product at every observation."""
    import torch
    p = workloads.ellipsoids_100x100x50()
    gold = np.load(os.path.join(HERE, "golden", "ellipsoids_100x100x50_rows.npz"))
    mesh, obs = _dev(g, p)
    v = np.abs(p.probe_v)
    w = _t(workloads.depth_weights(p.mesh, 25.0))
    for prec_name, tol in (("GRAV_MIXED", TOL_MIXED), ("GRAV_FP64", TOL_F64)):
        prec = getattr(g, prec_name)
        d = to_np(ctx.forward(mesh, obs, _t(p.m), prec=prec))
        err = rel_l2(d[gold["rows"]], gold["d"])
        _report(f"ellipsoids_100x100x50 forward {prec_name} (256 rows)", err)
        assert err <= tol
        gt = to_np(ctx.adjoint(mesh, obs, _t(v), prec=prec))
        got, ref = gt[gold["cells"]], gold["gtv"]
        if prec_name == "GRAV_FP64":
            # corner terms ~R ln R, each within a few ulp: C_TERMS * eps64 * sum |terms|
            _check_termwise(f"ellipsoids_100x100x50 adjoint {prec_name} (64 cells)", got, ref,
                            gold["gtv_abs_corners"], eps=2.0 ** -53,
                            rel_cap=_f64_corner_cap(ref, gold["gtv_abs_corners"]))
        else:
            _check_termwise(f"ellipsoids_100x100x50 adjoint {prec_name} (64 cells)", got, ref,
                            gold["gtv_abs"])
        diag = torch.empty(p.obs.n, dtype=torch.float64, device="cuda")
        tr = ctx.trace(mesh, obs, w, diag=diag, prec=prec)
        err = rel_l2(to_np(diag), gold["diag"])
        _report(f"ellipsoids_100x100x50 trace diagonal {prec_name} (10,000 rows)", err)
        assert err <= tol and abs(tr - float(gold["trace"])) <= tol * float(gold["trace"])
        out = to_np(ctx.dataspace_apply(mesh, obs, w, float(gold["ds_lambda"]), _t(v), prec=prec))
        err = rel_l2(out, gold["ds_out"])
        _report(f"ellipsoids_100x100x50 data-space {prec_name} (10,000 rows)", err)
        assert err <= tol


def test_paper_scale_forward_sampled_rows(g, ctx):
    """Paper-scale operators (178,797 x 3,307,500) in the launch configuration
    the benchmark times: G m on 2,000 stored oracle rows, G^T v (v = |probe|)
    on 48 stored cells, the data-space product for a probe on 64 stations on
    2,064 stored rows, and the diagonal of G C G^T at those 64 stations."""
    import torch
    p = workloads.paper_scale()
    gold = np.load(os.path.join(HERE, "golden", "paper_scale_rows.npz"))
    mesh, obs = _dev(g, p)
    d = to_np(ctx.forward(mesh, obs, _t(p.m), prec=g.GRAV_MIXED))
    err = rel_l2(d[gold["rows"]], gold["d"])
    _report("paper_scale forward GRAV_MIXED (2000 rows)", err)
    assert err <= TOL_MIXED
    gt = to_np(ctx.adjoint(mesh, obs, _t(np.abs(p.probe_v)), prec=g.GRAV_MIXED))
    _check_termwise("paper_scale adjoint GRAV_MIXED (48 cells)", gt[gold["cells"]], gold["gtv"],
                    gold["gtv_abs"])
    v = np.zeros(p.obs.n)
    v[gold["ds_support"]] = gold["ds_v"]
    out = to_np(ctx.dataspace_apply(mesh, obs, _t(p.wdepth), float(gold["ds_lambda"]), _t(v),
                                    prec=g.GRAV_MIXED))
    err = rel_l2(out[gold["ds_rows"]], gold["ds_out"])
    _report("paper_scale data-space GRAV_MIXED (2,064 rows)", err)
    assert err <= TOL_MIXED
    diag = torch.empty(p.obs.n, dtype=torch.float64, device="cuda")
    ctx.trace(mesh, obs, _t(p.wdepth), diag=diag, prec=g.GRAV_MIXED)
    err = rel_l2(to_np(diag)[gold["ds_support"]], gold["ds_diag"])
    _report("paper_scale trace diagonal GRAV_MIXED (64 rows)", err)
    assert err <= TOL_MIXED


def test_paper_scale_adjoint_fp64_sampled_cells(g, ctx):
    """The plain FP64 adjoint at paper scale on the same 48 stored cells."""
    p = workloads.paper_scale()
    gold = np.load(os.path.join(HERE, "golden", "paper_scale_rows.npz"))
    mesh, obs = _dev(g, p)
    gt = to_np(ctx.adjoint(mesh, obs, _t(np.abs(p.probe_v)), prec=g.GRAV_FP64))
    _check_termwise("paper_scale adjoint GRAV_FP64 (48 cells)", gt[gold["cells"]], gold["gtv"],
                    gold["gtv_abs_corners"], eps=2.0 ** -53,
                    rel_cap=_f64_corner_cap(gold["gtv"], gold["gtv_abs_corners"]))


# ------------------------------------------------------------------ multi-model

# Per-model relative L2 of the split-bf16 / FP32 G-tile contraction.  The
# three-product split keeps G m to about 3 x 2^-18 = 1.1e-5 of each term
# (bf16 hi + lo represent G and m to 2^-18 each; the dropped lo x lo product is
# below 2^-18 of the term); G_ok >= 0 below the stations, so with these
# models' moderate cancellation the per-model error stays well inside that
# (measured <= 2.9e-6, on the 4 x 4 x 2 single-model case).
TOL_MULTI = 1e-5


def _blocky_models(mesh, K, seed):
    rng = np.random.default_rng(seed)
    wx = mesh.xn[-1] - mesh.xn[0]
    cols = [workloads.ellipsoid_model(mesh, rng, 3, 0.1 * wx, 0.6 * wx) + 20.0 * rng.standard_normal(mesh.ncells)
            for _ in range(K)]
    return np.ascontiguousarray(np.stack(cols, axis=1).astype(np.float32))


@pytest.mark.parametrize("prec_name", ["GRAV_MIXED_BF16X3", "GRAV_FP32_VALU"])
@pytest.mark.parametrize("case", [
    dict(seed=21, nx=9, ny=6, nz=5, n=130, K=5),
    dict(seed=22, nx=17, ny=13, nz=11, n=70, K=64),
    dict(seed=23, nx=4, ny=4, nz=2, n=64, K=1),
    # one layer: the kernel's only layer step holds a single layer
    dict(seed=25, nx=6, ny=5, nz=1, n=80, K=3),
    # 23 layers, first deep layer 12: general and deep layer pairs, and a last
    # step with one deep layer
    dict(seed=27, nx=7, ny=6, nz=23, n=100, K=64),
])
def test_forward_multi_per_model(g, ctx, prec_name, case):
    import torch
    p = workloads.random_case(case["seed"], case["nx"], case["ny"], case["nz"], case["n"], on_top=10,
                              on_nodes=5)
    models = _blocky_models(p.mesh, case["K"], case["seed"])
    mesh, obs = _dev(g, p)
    D = to_np(ctx.forward_multi(mesh, obs, torch.as_tensor(models, device="cuda"),
                                prec=getattr(g, prec_name)))
    ref = prism.forward_multi(p.mesh, p.obs, models.astype(np.float64))
    errs = np.linalg.norm(D - ref, axis=0) / np.linalg.norm(ref, axis=0)
    print(f"[parity] multi {prec_name} {case}: per-model rel L2 max {errs.max():.2e} "
          f"median {np.median(errs):.2e}", flush=True)
    assert np.all(errs <= TOL_MULTI)


def test_forward_multi_chunks_of_several_blocks(g, ctx):
    """Enough observations (33,000) that each chunk of the prism-column blocks
    holds several blocks, so consecutive blocks share an edge row; the mesh is
    ragged in x and y (18 x 15 cells: partial blocks) and chunks start in the
    middle of a block row.  200 seeded rows per model against the oracle."""
    import torch
    p = workloads.random_case(24, 18, 15, 7, 33_000, on_top=40, on_nodes=20)
    models = _blocky_models(p.mesh, 7, 24)
    rows = np.sort(np.random.default_rng(24).choice(p.obs.n, 200, replace=False))
    ref = prism.forward_multi(p.mesh, p.obs, models.astype(np.float64), rows=rows)
    mesh, obs = _dev(g, p)
    mt = torch.as_tensor(models, device="cuda")
    for prec_name in ("GRAV_MIXED_BF16X3", "GRAV_FP32_VALU"):
        D = to_np(ctx.forward_multi(mesh, obs, mt, prec=getattr(g, prec_name)))[rows]
        errs = np.linalg.norm(D - ref, axis=0) / np.linalg.norm(ref, axis=0)
        print(f"[parity] multi chunks of several blocks {prec_name}: per-model rel L2 max "
              f"{errs.max():.2e} median {np.median(errs):.2e}", flush=True)
        assert np.all(errs <= TOL_MULTI)


def test_forward_multi_box_models_sampled_rows(g, ctx):
    """64 models on the 500k-cell mesh with 10,000 observations; 48 seeded rows
    per model against the FP64 oracle, for both contraction paths."""
    import torch
    p = workloads.ellipsoids_100x100x50()
    models = workloads.smoothed_box_models(p.mesh).astype(np.float32)
    rows = np.sort(np.random.default_rng(333).choice(p.obs.n, 48, replace=False))
    ref = prism.forward_multi(p.mesh, p.obs, models.astype(np.float64), rows=rows)
    mesh, obs = _dev(g, p)
    mt = torch.as_tensor(models, device="cuda")
    for prec_name in ("GRAV_MIXED_BF16X3", "GRAV_FP32_VALU"):
        D = to_np(ctx.forward_multi(mesh, obs, mt, prec=getattr(g, prec_name)))[rows]
        errs = np.linalg.norm(D - ref, axis=0) / np.linalg.norm(ref, axis=0)
        print(f"[parity] box models multi {prec_name}: per-model rel L2 max {errs.max():.2e} "
              f"median {np.median(errs):.2e}", flush=True)
        assert np.all(errs <= TOL_MULTI)


# ------------------------------------------------------------------ determinism and errors

def test_bitwise_repeatable(g, ctx):
    p = workloads.random_case(12, 20, 20, 10, 300)
    mesh, obs = _dev(g, p)
    for prec in (g.GRAV_MIXED, g.GRAV_FP64):
        a = to_np(ctx.forward(mesh, obs, _t(p.m), prec=prec))
        b = to_np(ctx.forward(mesh, obs, _t(p.m), prec=prec))
        assert np.array_equal(a, b)
        a = to_np(ctx.adjoint(mesh, obs, _t(p.probe_v), prec=prec))
        b = to_np(ctx.adjoint(mesh, obs, _t(p.probe_v), prec=prec))
        assert np.array_equal(a, b)


def test_error_paths(g, ctx):
    import torch
    p = workloads.random_case(13, 4, 4, 3, 10)
    mesh, obs = _dev(g, p)
    m = _t(p.m)
    # observation below the mesh top
    bad = g.DeviceObs(p.obs.x, p.obs.y, p.obs.z + 1e3)
    with pytest.raises(g.GravError) as e:
        ctx.forward(mesh, bad, m)
    assert e.value.code == g.GRAV_EINVAL and "below" in str(e.value)
    # non-increasing nodes
    xn = p.mesh.xn.copy()
    xn[2] = xn[1]
    badmesh = g.DeviceMesh(xn, p.mesh.yn, p.mesh.zn)
    with pytest.raises(g.GravError) as e:
        ctx.forward(badmesh, obs, m)
    assert e.value.code == g.GRAV_EINVAL
    # non-positive depth weight
    w = p.wdepth.copy()
    w[3] = 0.0
    with pytest.raises(g.GravError) as e:
        ctx.dataspace_apply(mesh, obs, _t(w), 1.0, _t(p.probe_v))
    assert e.value.code == g.GRAV_EINVAL
    # negative lambda for the operator
    with pytest.raises(g.GravError):
        ctx.dataspace_apply(mesh, obs, _t(p.wdepth), -1.0, _t(p.probe_v))
    # NULL pointers straight through the C ABI
    import ctypes
    rc = g.lib.grav_forward(ctx.handle, ctypes.byref(mesh.c), ctypes.byref(obs.c), None, None,
                            g.GRAV_MIXED, None)
    assert rc == g.GRAV_EINVAL
    # workspace too small
    small = g.Context(device=0, workspace_bytes=256)
    with pytest.raises(g.GravError) as e:
        small.forward(mesh, obs, m)
    assert e.value.code == g.GRAV_ENOMEM
    small.close()
    # unsupported precision for the operator
    with pytest.raises(g.GravError):
        ctx.forward(mesh, obs, m, prec=g.GRAV_MIXED_BF16X3)
    # empty inputs: no observations, a mesh without layers
    d = torch.empty(p.obs.n, dtype=torch.float64, device="cuda")
    empty_obs = g.CObs(0, None, None, None)
    rc = g.lib.grav_forward(ctx.handle, ctypes.byref(mesh.c), ctypes.byref(empty_obs), m.data_ptr(),
                            d.data_ptr(), g.GRAV_MIXED, None)
    assert rc == g.GRAV_EINVAL and b"positive" in g.lib.grav_last_error(ctx.handle)
    flat = g.CMesh(p.mesh.nx, p.mesh.ny, 0, mesh.c.xn, mesh.c.yn, mesh.c.zn)
    rc = g.lib.grav_forward(ctx.handle, ctypes.byref(flat), ctypes.byref(obs.c), m.data_ptr(),
                            d.data_ptr(), g.GRAV_MIXED, None)
    assert rc == g.GRAV_EINVAL
    # an observation beyond the validated range (node distance above 1e6 m)
    far = g.DeviceObs(p.obs.x + 2e6, p.obs.y, p.obs.z)
    with pytest.raises(g.GravError) as e:
        ctx.forward(mesh, far, m)
    assert e.value.code == g.GRAV_EINVAL and "1e6" in str(e.value)
    # the context is still usable after every rejection
    ok = ctx.forward(mesh, obs, m, prec=g.GRAV_FP64)
    assert rel_l2(to_np(ok), prism.forward(p.mesh, p.obs, p.m)) <= 1e-10
    torch.cuda.synchronize()


def test_forward_accuracy_over_and_around_the_mesh(g, ctx):
    """Per-station accuracy where the surveys of the method put stations: over
    the mesh footprint and up to half its width beyond it, 0-50 m above the
    top.  With a positive density every gz is a sum without cancellation
    between cells, so each station is checked to the relative tolerance of
    GRAV_MIXED on its own."""
    rng = np.random.default_rng(78)
    mesh = workloads.regular_mesh(12, 10, 8, 50.0, 50.0, 50.0)
    n = 400
    obs = workloads.Survey(rng.uniform(-300.0, 900.0, n), rng.uniform(-250.0, 750.0, n),
                           -rng.uniform(0.0, 50.0, n))
    m = rng.uniform(100.0, 400.0, mesh.ncells)
    dm, do = g.DeviceMesh.from_mesh(mesh), g.DeviceObs.from_survey(obs)
    d = to_np(ctx.forward(dm, do, _t(m), prec=g.GRAV_MIXED))
    ref = prism.forward(mesh, obs, m)
    rel = np.abs(d - ref) / np.abs(ref)
    print(f"[parity] stations over and around the mesh GRAV_MIXED: max rel {rel.max():.2e}, "
          f"rel L2 {rel_l2(d, ref):.2e}", flush=True)
    assert np.all(ref > 0) and np.all(rel <= TOL_MIXED)


def test_forward_far_field_is_finite_within_rounding_scale(g, ctx):
    """Stations up to 0.89e6 m from a 600 m mesh, inside the 1e6 m range the
    library accepts.  There the edge terms of a far station cancel by
    ~(R/L)^2 (R/L up to ~1.5e3), so GRAV_MIXED's relative accuracy is lost
    (GRAV_FP64 is the path for such stations); what is claimed and checked is
    that every result is finite and within the rounding scale of the terms it
    adds: |error| <= 16 eps32 x (sum of |S W2| over the segments, the oracle's
    forward_abs_scale)."""
    rng = np.random.default_rng(77)
    mesh = workloads.regular_mesh(6, 5, 4, 100.0, 100.0, 100.0)
    n = 48
    r = rng.uniform(1e3, 8.9e5, n)
    th = rng.uniform(0, 2 * np.pi, n)
    obs = workloads.Survey(300.0 + r * np.cos(th), 250.0 + r * np.sin(th), -rng.uniform(0, 50, n))
    m = rng.uniform(-300, 300, mesh.ncells)
    dm, do = g.DeviceMesh.from_mesh(mesh), g.DeviceObs.from_survey(obs)
    d = to_np(ctx.forward(dm, do, _t(m), prec=g.GRAV_MIXED))
    ref = prism.forward(mesh, obs, m)
    scale = prism.forward_abs_scale(mesh, obs, m, np.arange(n))
    ratio = np.abs(d - ref) / (16 * 2.0 ** -24 * scale)
    print(f"[parity] far field to 0.89e6 m GRAV_MIXED: worst err / term bound = {ratio.max():.3f}",
          flush=True)
    assert np.all(np.isfinite(d)) and np.all(ratio <= 1.0)


# ------------------------------------------------------------------ trend surface

def _regional_field(seed, n):
    """Stations over a 128 km x 220 km block (the extent of the regional
    survey) with a second-degree regional trend plus local anomalies and noise."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.28e5, n) + 3.0e5
    y = rng.uniform(0.0, 2.2e5, n) + 2.6e6
    u, w = (x - 3.64e5) / 1e5, (y - 2.71e6) / 1e5
    regional = 4e-4 - 2e-4 * u + 1e-4 * w + 5e-5 * u * u - 8e-5 * u * w + 3e-5 * w * w
    local = sum(a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * s * s))
                for a, cx, cy, s in zip(rng.normal(0, 2e-5, 12), rng.uniform(3e5, 4.28e5, 12),
                                        rng.uniform(2.6e6, 2.82e6, 12), rng.uniform(2e3, 1.5e4, 12)))
    return x, y, regional + local + 1e-6 * rng.standard_normal(n)


@pytest.mark.parametrize("n,degree", [(7, 2), (1000, 1), (178797, 2)])
def test_trend_surface_vs_oracle(g, ctx, n, degree):
    import torch
    x, y, v = _regional_field(50 + n, n)
    t_ref, r_ref = trend_oracle.trend_surface(x, y, v, degree)
    tx, ty, tv = _t(x), _t(y), _t(v)
    resid = torch.empty_like(tv)
    tr = torch.empty_like(tv)
    coef, frame = ctx.trend_surface(tx, ty, tv, degree, resid=resid, trend=tr)
    print(f"[parity] trend n={n} degree={degree}: frame {frame}", flush=True)
    scale = np.abs(t_ref).max()
    np.testing.assert_allclose(to_np(tr), t_ref, rtol=0, atol=1e-9 * scale)
    np.testing.assert_allclose(to_np(resid), r_ref, rtol=0, atol=1e-9 * scale)
    # the returned coefficients and frame describe the same surface
    u, w = (x - frame[0]) / frame[2], (y - frame[1]) / frame[2]
    host = np.stack([np.ones_like(u), u, w, u * u, u * w, w * w], 1) @ np.asarray(coef)
    np.testing.assert_allclose(host, t_ref, rtol=0, atol=1e-9 * scale)
    if degree == 1:
        assert coef[3:] == [0.0, 0.0, 0.0]
    # residual in place, bitwise equal to the separate output
    tv2 = tv.clone()
    ctx.trend_surface(tx, ty, tv2, degree, resid=tv2)
    assert torch.equal(tv2, resid)


def test_trend_surface_errors(g, ctx):
    import torch
    x, y, v = _regional_field(9, 40)
    tx, ty, tv = _t(x), _t(y), _t(v)
    with pytest.raises(g.GravError):
        ctx.trend_surface(tx, ty, tv, 3)
    with pytest.raises(g.GravError):
        ctx.trend_surface(tx[:5], ty[:5], tv[:5], 2)
    with pytest.raises(g.GravError):      # collinear stations do not fix a quadratic
        ctx.trend_surface(torch.full_like(tx, 3e5), ty, tv, 2)
    bad = tv.clone()
    bad[17] = float("nan")
    with pytest.raises(g.GravError):
        ctx.trend_surface(tx, ty, bad, 2)
    coef, frame = ctx.trend_surface(tx, ty, tv, 2)     # the context still works
    assert np.all(np.isfinite(coef))
