"""GPU tests of the continuous-batching server: a request's result is the
same (bitwise) alone and in a mix, equals the single-call operators, memory
admission queues instead of failing, and bad requests are rejected."""
import time

import numpy as np
import pytest

import workloads
from oracle import prism, inversion
from tests._util import load_package, rel_l2, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    pkg = load_package()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return pkg


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _requests():
    """A mix of uneven shapes: forward and inversion problems."""
    cases = []
    for seed, (nx, ny, nz, n, kind) in enumerate([(14, 12, 6, 300, "inv"), (20, 9, 11, 77, "fwd"),
                                                   (8, 8, 8, 130, "inv"), (31, 17, 5, 500, "fwd"),
                                                   (10, 12, 7, 64, "inv")]):
        p = workloads.random_case(100 + seed, nx, ny, nz, n, model="blocky", on_top=n // 5)
        cases.append((kind, p))
    return cases


def _device_problem(g, kind, p):
    import torch
    mesh, obs = g.DeviceMesh.from_mesh(p.mesh), g.DeviceObs.from_survey(p.obs)
    if kind == "fwd":
        return dict(mesh=mesh, obs=obs, m=_t(p.m), d=torch.empty(p.obs.n, dtype=torch.float64, device="cuda"))
    d_clean = prism.forward(p.mesh, p.obs, p.m)
    d_obs = inversion.add_noise(d_clean, p.noise_draws, 0.01)
    return dict(mesh=mesh, obs=obs, d_obs=_t(d_obs), w=_t(p.wdepth),
                m_out=torch.empty(p.mesh.ncells, dtype=torch.float64, device="cuda"))


def _submit(srv, kind, dp, tol=1e-8, max_iter=300):
    if kind == "fwd":
        return srv.submit_forward(dp["mesh"], dp["obs"], dp["m"], dp["d"])
    return srv.submit_invert(dp["mesh"], dp["obs"], dp["d_obs"], dp["w"], dp["m_out"], lam=-1.0,
                             tol=tol, max_iter=max_iter)


def _result(kind, dp):
    return to_np(dp["d"] if kind == "fwd" else dp["m_out"]).copy()


def test_results_identical_alone_and_in_mix(g):
    cases = _requests()
    alone = []
    with g.Server(0, budget_bytes=1 << 30) as srv:
        for kind, p in cases:
            dp = _device_problem(g, kind, p)
            info = srv.wait(_submit(srv, kind, dp))
            alone.append((_result(kind, dp), info))
        mixed = [_device_problem(g, kind, p) for kind, p in cases]
        tickets = [_submit(srv, kind, dp) for (kind, _), dp in zip(cases, mixed)]
        infos = [srv.wait(t) for t in tickets]
    for (kind, _), dp, (ref, info_a), info_m in zip(cases, mixed, alone, infos):
        assert np.array_equal(_result(kind, dp), ref), kind
        assert info_a["iters"] == info_m["iters"]
        print(f"[serving] {kind}: iters {info_m['iters']} relres {info_m['relres']:.2e} "
              f"queue {info_m['queue_ms']:.1f} ms run {info_m['run_ms']:.1f} ms", flush=True)


def test_served_equals_single_call_operators(g):
    import torch
    cases = _requests()
    ctx = g.Context(0)
    with g.Server(0, budget_bytes=1 << 30) as srv:
        dps = [_device_problem(g, kind, p) for kind, p in cases]
        tickets = [_submit(srv, kind, dp) for (kind, _), dp in zip(cases, dps)]
        infos = [srv.wait(t) for t in tickets]
    for (kind, p), dp, info in zip(cases, dps, infos):
        if kind == "fwd":
            d = ctx.forward(dp["mesh"], dp["obs"], dp["m"], prec=g.GRAV_MIXED)
            assert torch.equal(d, dp["d"])
            assert rel_l2(to_np(d), prism.forward(p.mesh, p.obs, p.m)) <= 1e-5
        else:
            m, _, inf = ctx.invert(dp["mesh"], dp["obs"], dp["d_obs"], dp["w"], lam=-1.0, tol=1e-8,
                                   max_iter=300, prec=g.GRAV_MIXED)
            assert inf["iters"] == info["iters"]
            assert abs(inf["lambda_used"] - info["lambda_used"]) <= 1e-12 * inf["lambda_used"]
            assert torch.equal(m, dp["m_out"])
    ctx.close()


def test_admission_by_memory_queues_instead_of_failing(g):
    cases = _requests()
    with g.Server(0, budget_bytes=1 << 30) as probe:
        sizes = []
        for kind, p in cases:
            dp = _device_problem(g, kind, p)
            sizes.append(probe.wait(_submit(probe, kind, dp))["state_bytes"])
    budget = max(sizes) + 4096          # room for the largest request, rarely for two
    with g.Server(0, budget_bytes=budget) as srv:
        dps = [_device_problem(g, kind, p) for kind, p in cases]
        tickets = [_submit(srv, kind, dp) for (kind, _), dp in zip(cases, dps)]
        infos = [srv.wait(t) for t in tickets]
    assert all(i["status"] in (0, 4) for i in infos)
    assert max(i["queue_ms"] for i in infos) > 0.0


def test_bad_requests_rejected(g):
    import torch
    p = workloads.random_case(7, 5, 5, 4, 20)
    with g.Server(0, budget_bytes=64 << 20) as srv:
        bad_obs = g.DeviceObs(p.obs.x, p.obs.y, p.obs.z + 1e4)
        mesh = g.DeviceMesh.from_mesh(p.mesh)
        d = torch.empty(p.obs.n, dtype=torch.float64, device="cuda")
        with pytest.raises(g.GravError) as e:
            srv.submit_forward(mesh, bad_obs, _t(p.m), d)
        assert e.value.code == g.GRAV_EINVAL
        big = workloads.random_case(8, 120, 120, 60, 4000)
        bm, bo = g.DeviceMesh.from_mesh(big.mesh), g.DeviceObs.from_survey(big.obs)
        with pytest.raises(g.GravError) as e:
            srv.submit_invert(bm, bo, _t(np.ones(big.obs.n)), _t(big.wdepth),
                              torch.empty(big.mesh.ncells, dtype=torch.float64, device="cuda"))
        assert e.value.code == g.GRAV_ENOMEM
        # the server still works after rejections
        obs = g.DeviceObs.from_survey(p.obs)
        t = srv.submit_forward(mesh, obs, _t(p.m), d)
        srv.wait(t)
        assert rel_l2(to_np(d), prism.forward(p.mesh, p.obs, p.m)) <= 1e-5


def test_forward_requests_pass_inversions_waiting_for_a_slot(g):
    """With one inversion slot, a forward request submitted behind a queued
    inversion is served while the first inversion runs; the queued inversion
    starts only when the slot frees."""
    cases = _requests()
    (ka, pa), (kc, pc), (kb, pb) = cases[0], cases[1], cases[2]
    assert (ka, kc, kb) == ("inv", "fwd", "inv")
    with g.Server(0, max_active=1, budget_bytes=1 << 30) as srv:
        da, db, dc = (_device_problem(g, k, p) for k, p in ((ka, pa), (kb, pb), (kc, pc)))
        ta = _submit(srv, ka, da)
        tb = _submit(srv, kb, db)
        tc = _submit(srv, kc, dc)
        ia, ib, ic = srv.wait(ta), srv.wait(tb), srv.wait(tc)
    print(f"[serving] one slot: A run {ia['run_ms']:.1f} ms, B queue {ib['queue_ms']:.1f} ms, "
          f"C queue {ic['queue_ms']:.1f} ms run {ic['run_ms']:.1f} ms", flush=True)
    assert ia["iters"] > 10
    # C finished before A did; B waited for A's slot
    assert ic["queue_ms"] + ic["run_ms"] < ia["queue_ms"] + ia["run_ms"]
    assert ib["queue_ms"] >= 0.9 * (ia["queue_ms"] + ia["run_ms"])
    assert rel_l2(_result(kc, dc), prism.forward(pc.mesh, pc.obs, pc.m)) <= 1e-5


def test_serving_stream_largest_requests_sampled():
    """The largest forward request of the serving stream (about 40k stations
    over about 800k cells) served in a mix with stream inversions: its data
    match the FP64 oracle on sampled stations, and the inversions finish."""
    import torch
    pkg = load_package()
    reqs = workloads.serving_stream()
    fwd = max((r for r in reqs if r["kind"] == "forward"),
              key=lambda r: r["n_target"] * r["cells_target"])
    invs = sorted((r for r in reqs if r["kind"] == "inversion"),
                  key=lambda r: r["n_target"] * r["cells_target"])[:3]
    pf = fwd["build"]()
    print(f"[serving] largest forward: {pf.obs.n} stations x {pf.mesh.ncells} cells", flush=True)
    mesh, obs = pkg.DeviceMesh.from_mesh(pf.mesh), pkg.DeviceObs.from_survey(pf.obs)
    d = torch.empty(pf.obs.n, dtype=torch.float64, device="cuda")
    with pkg.Server(0, budget_bytes=8 << 30) as srv:
        items = []
        for r in invs:
            p = r["build"]()
            dm, do = pkg.DeviceMesh.from_mesh(p.mesh), pkg.DeviceObs.from_survey(p.obs)
            d_obs = _t(inversion.add_noise(prism.forward(p.mesh, p.obs, p.m), p.noise_draws,
                                           p.noise_level))
            m_out = torch.empty(p.mesh.ncells, dtype=torch.float64, device="cuda")
            items.append((dm, do, d_obs, m_out))
            srv_t = srv.submit_invert(dm, do, d_obs, _t(p.wdepth), m_out, lam=-1.0,
                                      tol=p.cg_tol, max_iter=p.cg_iters)
            items[-1] += (srv_t,)
        tf = srv.submit_forward(mesh, obs, _t(pf.m), d)
        info_f = srv.wait(tf)
        infos = [srv.wait(it[-1]) for it in items]
    rows = np.sort(np.random.default_rng(55).choice(pf.obs.n, 16, replace=False))
    ref = prism.forward(pf.mesh, pf.obs, pf.m, rows)
    err = rel_l2(to_np(d)[rows], ref)
    print(f"[serving] largest forward, 16 sampled stations: rel L2 = {err:.3e}; inversions "
          f"{[i['iters'] for i in infos]} iterations, status {[i['status'] for i in infos]}",
          flush=True)
    assert info_f["status"] == 0 and err <= 1e-5
    assert all(i["status"] in (0, 4) for i in infos)
    assert all(np.all(np.isfinite(to_np(it[3]))) for it in items)


def test_cancel_queued_and_running_requests(g):
    """Cancelling a queued inversion drops it at once; cancelling a running one
    stops it after the current step; both report GRAV_ECANCELED, and the
    server keeps serving (a later request equals the single-call result)."""
    import torch
    cases = _requests()
    (ka, pa), (kb, pb) = cases[0], cases[2]
    ctx = g.Context(0)
    with g.Server(0, max_active=1, budget_bytes=1 << 30) as srv:
        da, db = _device_problem(g, ka, pa), _device_problem(g, kb, pb)
        ta = srv.submit_invert(da["mesh"], da["obs"], da["d_obs"], da["w"], da["m_out"],
                               lam=-1.0, fixed_iters=1_000_000)  # runs until cancelled
        tb = _submit(srv, kb, db)                                # waits for the one slot
        srv.cancel(tb)
        ib = srv.wait(tb)
        assert ib["status"] == g.GRAV_ECANCELED and ib["run_ms"] == 0.0
        time.sleep(0.3)                                          # let A run some steps
        srv.cancel(ta)
        ia = srv.wait(ta)
        assert ia["status"] == g.GRAV_ECANCELED and 0 < ia["iters"] < 1_000_000
        with pytest.raises(g.GravError):
            srv.cancel(ta)                                       # retired ticket
        dc = _device_problem(g, kb, pb)
        ic = srv.wait(_submit(srv, kb, dc))
        assert ic["status"] == 0
    m, _, inf = ctx.invert(dc["mesh"], dc["obs"], dc["d_obs"], dc["w"], lam=-1.0, tol=1e-8,
                           max_iter=300, prec=g.GRAV_MIXED)
    assert inf["iters"] == ic["iters"] and torch.equal(m, dc["m_out"])
    ctx.close()
    print(f"[serving] cancel: running request stopped after {ia['iters']} iterations", flush=True)


def test_concurrent_submission_from_threads(g):
    """Requests submitted from several threads at once are all served, each
    bitwise equal to its single-call result."""
    import threading
    import torch
    ctx = g.Context(0)
    cases = [workloads.random_case(300 + i, 9 + i, 7, 5, 90 + 13 * i, model="blocky")
             for i in range(8)]
    refs = [ctx.forward(g.DeviceMesh.from_mesh(p.mesh), g.DeviceObs.from_survey(p.obs), _t(p.m),
                        prec=g.GRAV_MIXED) for p in cases]
    outs = [torch.empty(p.obs.n, dtype=torch.float64, device="cuda") for p in cases]
    errors = []
    with g.Server(0, max_active=4, budget_bytes=1 << 30) as srv:
        def client(idx):
            try:
                p = cases[idx]
                mesh, obs = g.DeviceMesh.from_mesh(p.mesh), g.DeviceObs.from_survey(p.obs)
                for _ in range(3):
                    info = srv.wait(srv.submit_forward(mesh, obs, _t(p.m), outs[idx]))
                    assert info["status"] == 0
            except Exception as e:  # noqa: BLE001  (reported below)
                errors.append(e)
        threads = [threading.Thread(target=client, args=(i,)) for i in range(len(cases))]
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=120)
    assert not errors, errors
    for ref, out in zip(refs, outs):
        assert torch.equal(ref, out)
    ctx.close()


def test_largest_slot_count_with_many_small_requests(g):
    """max_active at its cap (256): 300 small forward requests submitted at
    once are all served; a sample is bitwise equal to the single-call path."""
    import torch
    p = workloads.random_case(400, 6, 5, 4, 70, model="blocky")
    mesh, obs = g.DeviceMesh.from_mesh(p.mesh), g.DeviceObs.from_survey(p.obs)
    m = _t(p.m)
    with g.Context(0) as ctx:
        ref = ctx.forward(mesh, obs, m, prec=g.GRAV_MIXED)
    outs = [torch.empty(p.obs.n, dtype=torch.float64, device="cuda") for _ in range(300)]
    with g.Server(0, max_active=256, budget_bytes=1 << 30) as srv:
        tickets = [srv.submit_forward(mesh, obs, m, d) for d in outs]
        infos = [srv.wait(t) for t in tickets]
    assert all(i["status"] == 0 for i in infos)
    assert all(torch.equal(d, ref) for d in outs[::37])
    with pytest.raises(g.GravError):
        g.Server(0, max_active=257)


def test_inputs_produced_asynchronously_on_the_current_stream(g):
    """A request whose density is still being written on torch's current
    stream when it is submitted: submit orders the server's reads after that
    work, so the result equals the single-call forward of the final density."""
    import torch
    p = workloads.random_case(140, 24, 20, 9, 400, model="blocky", on_top=40)
    mesh, obs = g.DeviceMesh.from_mesh(p.mesh), g.DeviceObs.from_survey(p.obs)
    with g.Context(0) as ctx:
        ref = to_np(ctx.forward(mesh, obs, _t(p.m), prec=g.GRAV_MIXED))
    m_host = torch.as_tensor(p.m).pin_memory()
    side = torch.cuda.Stream()
    with g.Server(0, budget_bytes=1 << 28) as srv, torch.cuda.stream(side):
        # a queue of device work ahead of the copy that fills m
        a = torch.randn(2048, 2048, device="cuda")
        for _ in range(24):
            a = torch.tanh(a @ a * 1e-3)
        m = torch.empty(p.mesh.ncells, dtype=torch.float64, device="cuda")
        m.fill_(float("nan"))
        m.copy_(m_host, non_blocking=True)
        d = torch.empty(p.obs.n, dtype=torch.float64, device="cuda")
        info = srv.wait(srv.submit_forward(mesh, obs, m, d))
        assert info["status"] == g.GRAV_OK
        side.synchronize()
    assert np.array_equal(to_np(d), ref)
