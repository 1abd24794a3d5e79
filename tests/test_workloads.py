"""The seeded synthetic workloads match their stated recipes (CPU only):
sizes, ranges, seeds and determinism of the inputs every GPU test and the
benchmark are fed with."""
import math

import numpy as np
import pytest

import workloads


@pytest.fixture(scope="module")
def paper_scale():
    return workloads.paper_scale()


def test_paper_scale_recipe(paper_scale):
    p = paper_scale
    assert p.mesh.shape == (150, 150, 147) and p.mesh.ncells == 3_307_500
    assert np.allclose(np.diff(p.mesh.xn), 100.0) and np.allclose(np.diff(p.mesh.yn), 100.0)
    assert np.allclose(np.diff(p.mesh.zn), 70.0)
    assert p.obs.n == 178_797
    assert p.obs.x.min() >= 0.0 and p.obs.x.max() <= 15000.0
    assert p.obs.y.min() >= 0.0 and p.obs.y.max() <= 15000.0
    h = p.mesh.zn[0] - p.obs.z
    assert h.min() >= 0.0 and math.isclose(h.max(), 300.0)   # every station on or above the top
    assert p.m.max() >= 300.0 and np.count_nonzero(p.m) > 0
    assert p.noise_level == 0.02 and p.cg_iters == 50 and p.lambda_factor == 1e-2
    # w = (depth of the cell centre below the top + 25 m)^-1
    k = np.arange(147)
    assert np.allclose(p.wdepth.reshape(150, 150, 147)[3, 7], 1.0 / (70.0 * k + 35.0 + 25.0))


def test_paper_scale_is_deterministic(paper_scale):
    q = workloads.paper_scale()
    for a, b in ((paper_scale.obs.x, q.obs.x), (paper_scale.obs.z, q.obs.z),
                 (paper_scale.m, q.m), (paper_scale.noise_draws, q.noise_draws),
                 (paper_scale.probe_v, q.probe_v)):
        assert np.array_equal(a, b)


def test_ellipsoids_recipe():
    p = workloads.ellipsoids_100x100x50()
    assert p.mesh.shape == (100, 100, 50)
    assert np.allclose(np.diff(p.mesh.zn), 25.0)
    assert p.obs.n == 10_000
    xc = 12.5 + 25.0 * np.arange(100)
    assert np.allclose(np.unique(p.obs.x), xc) and np.allclose(np.unique(p.obs.y), xc)
    h = p.mesh.zn[0] - p.obs.z
    assert h.min() >= 0.0 and h.max() <= 50.0
    assert np.abs(p.m).max() > 0 and p.probe_v.shape == (10_000,)


def test_serving_stream_recipe():
    reqs = workloads.serving_stream()
    assert len(reqs) == 200
    t = np.array([r["t"] for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert 0.35 < np.mean(np.diff(t)) < 0.65                 # exponential gaps, mean 0.5 s
    kinds = [r["kind"] for r in reqs]
    assert set(kinds) == {"forward", "inversion"} and 60 < kinds.count("forward") < 140
    assert all(1000 <= r["n_target"] <= 40_000 for r in reqs)
    assert all(50_000 <= r["cells_target"] <= 800_000 for r in reqs)
    again = workloads.serving_stream()
    assert [r["seed"] for r in again] == [r["seed"] for r in reqs]


def test_serving_stream_request_shapes():
    reqs = workloads.serving_stream()
    for r in (reqs[0], min(reqs, key=lambda q: q["cells_target"])):
        p = r["build"]()
        nx, ny, nz = p.mesh.shape
        assert nx == ny == 2 * nz
        assert np.allclose(np.diff(p.mesh.zn), 25.0)
        assert abs(p.mesh.ncells - r["cells_target"]) <= 0.5 * r["cells_target"]
        g = round(math.sqrt(p.obs.n))
        assert g * g == p.obs.n and abs(p.obs.n - r["n_target"]) <= 2 * g + 1
        assert np.all(p.obs.z == p.mesh.zn[0])                 # stations on the mesh top
        assert p.noise_level == 0.01 and p.m.max() == 300.0
        assert p.cg_iters == (200 if r["kind"] == "inversion" else 0)
