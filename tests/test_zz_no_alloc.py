"""grav_forward_static (the forward product on the library's static device
scratch buffer, no context and no device allocation) against grav_forward on
the same inputs, through the C ABI: bitwise equal, and both within the
operator tolerance of the FP64 oracle.  Two calls in a row share the buffer;
the second has the smaller input, so stale contents of the first would show."""
import numpy as np
import pytest

from oracle import prism
import workloads
from tests._util import load_package, rel_l2, to_np

pytestmark = pytest.mark.gpu

TOL = {"GRAV_FP64": 1e-10, "GRAV_MIXED": 1e-5}


@pytest.fixture(scope="module")
def g():
    pkg = load_package()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return pkg


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


CASES = [
    # larger first, then smaller: the second call reuses what the first left
    dict(seed=41, nx=23, ny=17, nz=21, n=701, on_nodes=40, on_top=60),
    dict(seed=42, nx=6, ny=5, nz=3, n=37, on_nodes=5, on_top=5),
]


@pytest.mark.parametrize("validate", [1, 0])
@pytest.mark.parametrize("prec_name", ["GRAV_MIXED", "GRAV_FP64"])
def test_static_forward_matches_context_forward(g, prec_name, validate):
    import torch
    prec = getattr(g, prec_name)
    probs = [workloads.random_case(c["seed"], c["nx"], c["ny"], c["nz"], c["n"],
                                   on_nodes=c["on_nodes"], on_top=c["on_top"]) for c in CASES]
    with g.Context(0) as ctx:
        for case, p in zip(CASES, probs):
            print(f"[no-alloc] {prec_name} validate={validate} case {case}", flush=True)
            mesh = g.DeviceMesh.from_mesh(p.mesh)
            obs = g.DeviceObs.from_survey(p.obs)
            m = _t(p.m)
            d_static = g.forward_static(mesh, obs, m, prec=prec, validate=bool(validate))
            d_ctx = ctx.forward(mesh, obs, m, prec=prec)
            torch.cuda.synchronize()
            a, b = to_np(d_static), to_np(d_ctx)
            assert np.array_equal(a, b), f"max |diff| {np.max(np.abs(a - b)):.3e}"
            err = rel_l2(a, prism.forward(p.mesh, p.obs, p.m))
            print(f"[no-alloc] rel L2 vs oracle {err:.3e}", flush=True)
            assert err <= TOL[prec_name]


def test_static_forward_rejects_oversized_and_bad_arguments(g):
    import torch
    # 260 x 260 x 200 cells: the edge weights alone (261^2 * 200 doubles,
    # 104 MiB) and the partial sums exceed the 128 MiB buffer; rejected on
    # the host before anything is enqueued.
    nx, ny, nz, n = 260, 260, 200, 5000
    need = g.workspace_bytes(nx, ny, nz, n, g.OP_FORWARD, g.GRAV_MIXED) + 16384
    assert need > g.GRAV_STATIC_SCRATCH_BYTES
    mesh = g.DeviceMesh(np.arange(nx + 1) * 10.0, np.arange(ny + 1) * 10.0, np.arange(nz + 1) * 10.0)
    rng = np.random.default_rng(3)
    obs = g.DeviceObs(rng.uniform(0, 2600, n), rng.uniform(0, 2600, n), -rng.uniform(0, 50, n))
    m = torch.zeros(nx * ny * nz, dtype=torch.float64, device="cuda")
    with pytest.raises(g.GravError) as ei:
        g.forward_static(mesh, obs, m)
    assert ei.value.code == g.GRAV_ENOMEM
    assert "static buffer" in str(ei.value)
    # an observation below the mesh top: device validation rejects it
    p = workloads.random_case(7, 4, 4, 3, 10)
    bad_z = p.obs.z.copy()
    bad_z[3] = p.mesh.zn[0] + 1.0
    mesh2 = g.DeviceMesh.from_mesh(p.mesh)
    obs2 = g.DeviceObs(p.obs.x, p.obs.y, bad_z)
    with pytest.raises(g.GravError) as ei:
        g.forward_static(mesh2, obs2, _t(p.m))
    assert ei.value.code == g.GRAV_EINVAL
    # and a valid call on the same thread afterwards clears the error state
    d = g.forward_static(mesh2, g.DeviceObs.from_survey(p.obs), _t(p.m))
    assert rel_l2(to_np(d), prism.forward(p.mesh, p.obs, p.m)) <= 1e-5
