"""CG iterations replayed from a HIP graph (grav_cg_opts.graph = 1) against
the same solve with the kernels launched one by one: the same kernels with
the same arguments run in the same order, so the results are bitwise equal
(GPU against GPU, a property that holds at any size).  The graph is replayed
once per iteration with the solver's own host reads in between; the solves
are repeated with eager work between them and each is checked."""
import numpy as np
import pytest

from oracle import prism
import workloads
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


@pytest.fixture(scope="module")
def problems():
    out = []
    for p in (workloads.dykes_32x32x16(), workloads.random_case(31, 23, 19, 13, 700)):
        d = prism.forward(p.mesh, p.obs, p.m)
        out.append((p, d))
    return out


@pytest.mark.parametrize("prec_name", ["GRAV_MIXED", "GRAV_FP64"])
@pytest.mark.parametrize("precond", [0, 1])
def test_graph_replay_equals_eager(g, problems, prec_name, precond):
    prec = getattr(g, prec_name)
    with g.Context(0) as ctx:
        for p, d in problems:
            mesh, obs = g.DeviceMesh.from_mesh(p.mesh), g.DeviceObs.from_survey(p.obs)
            dd, w = _t(d), _t(p.wdepth)
            kw = dict(lam=-1.0, tol=1e-6, max_iter=300, prec=prec, precond=precond, history_cap=300)
            m0, _, i0 = ctx.invert(mesh, obs, dd, w, **kw)
            for rep in range(3):
                m1, _, i1 = ctx.invert(mesh, obs, dd, w, graph=True, **kw)
                print(f"[graph] {p.name} {prec_name} precond={precond} rep {rep}: {i1['iters']} "
                      f"iterations (eager {i0['iters']})", flush=True)
                assert i1["iters"] == i0["iters"] and i1["history"] == i0["history"]
                assert np.array_equal(to_np(m1), to_np(m0))
                # eager work on the same context between the replays
                ctx.forward(mesh, obs, m1, prec=prec)
            # fixed iteration count (no host read inside the loop)
            mf0, _, f0 = ctx.invert(mesh, obs, dd, w, lam=-1.0, fixed_iters=25, prec=prec,
                                    precond=precond)
            mf1, _, f1 = ctx.invert(mesh, obs, dd, w, lam=-1.0, fixed_iters=25, prec=prec,
                                    precond=precond, graph=True)
            assert f0["relres"] == f1["relres"] and np.array_equal(to_np(mf0), to_np(mf1))
            assert rel_l2(to_np(m0), to_np(mf0)) < 1.0


def test_graph_with_timing_and_errors(g, problems):
    p, d = problems[0]
    with g.Context(0) as ctx:
        mesh, obs = g.DeviceMesh.from_mesh(p.mesh), g.DeviceObs.from_survey(p.obs)
        dd, w = _t(d), _t(p.wdepth)
        m0, _, i0 = ctx.invert(mesh, obs, dd, w, tol=1e-6)
        ctx.set_timing(True)          # the graph is not used while timing is on
        m1, _, i1 = ctx.invert(mesh, obs, dd, w, tol=1e-6, graph=True)
        ctx.set_timing(False)
        assert i1["iters"] == i0["iters"] and np.array_equal(to_np(m1), to_np(m0))
        # the restarted policy ignores the flag
        m2, _, i2 = ctx.invert(mesh, obs, dd, w, tol=1e-4, restart=20, max_cycles=30)
        m3, _, i3 = ctx.invert(mesh, obs, dd, w, tol=1e-4, restart=20, max_cycles=30, graph=True)
        assert i2["iters"] == i3["iters"] and np.array_equal(to_np(m2), to_np(m3))
        import ctypes
        from paper_2602_03857_amd._lib import CgOpts, CgInfo
        cg = CgOpts(1e-6, 100, 0, 0, 0, 0, 0, 0, None, None, None, 2)
        m_out = _t(np.zeros(p.mesh.ncells))
        rc = g.lib.grav_invert(ctx.handle, ctypes.byref(mesh.c), ctypes.byref(obs.c), dd.data_ptr(),
                               w.data_ptr(), -1.0, None, ctypes.byref(cg), m_out.data_ptr(), None,
                               ctypes.byref(CgInfo()), g.GRAV_MIXED, None)
        assert rc == g.GRAV_EINVAL and b"graph" in g.lib.grav_last_error(ctx.handle)
