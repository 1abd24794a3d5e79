"""Pins of the section-workflow oracle (``oracle.sections``; paper Section
4.5 with the trend separation of Section 2.2).  CPU only.

Each check ties the oracle to something other than itself: the plain
inversion it reduces to with one section, the model-space optimality
condition of Eq. 8 (a different form of the solve than the Cholesky of
Eq. 11 the oracle uses), exact recovery of planted polynomial trends, and
brute-force bookkeeping of the section split."""
import numpy as np
import pytest

from oracle import inversion, prism, sections, trend
import workloads


def _regional(seed=3, nx=6, ny=9, nz=4, n=72):
    """A small regional problem: two blocky bodies plus a second-degree
    regional field, 1 % noise."""
    p = workloads.random_case(seed, nx, ny, nz, n, model="blocky", on_top=n // 4)
    d = prism.forward(p.mesh, p.obs, p.m)
    u = (p.obs.x - p.obs.x.mean()) / 100.0
    w = (p.obs.y - p.obs.y.mean()) / 100.0
    regional = (2.0 + 0.7 * u - 0.4 * w + 0.3 * u * u - 0.2 * u * w + 0.1 * w * w) * np.abs(d).max()
    d_obs = inversion.add_noise(d + regional, p.noise_draws, 0.01)
    return p, d_obs, regional


def test_station_assignment_brute_force():
    p, _, _ = _regional()
    ysplit = [0, 3, 6, 9]
    sec = sections.section_of_stations(p.mesh, p.obs, ysplit)
    for o in range(p.obs.n):
        y = p.obs.y[o]
        want = 0
        for s in range(1, 3):
            if y >= p.mesh.yn[ysplit[s]]:
                want = s
        assert sec[o] == want
    # a station exactly on an interior boundary belongs to the section above it
    on = workloads.Survey(np.array([10.0]), np.array([p.mesh.yn[3]]), np.array([p.mesh.zn[0]]))
    assert sections.section_of_stations(p.mesh, on, ysplit)[0] == 1


def test_cell_slices_partition_the_mesh_in_section_order():
    mesh = workloads.regular_mesh(3, 7, 2, 10.0, 10.0, 10.0)
    ysplit = [0, 2, 5, 7]
    seen = np.concatenate([sections.cell_slice(mesh, ysplit[s], ysplit[s + 1]) for s in range(3)])
    assert np.array_equal(np.sort(seen), np.arange(mesh.ncells))
    # section cell (i, j', k) is regional cell (i, j0 + j', k)
    sl = sections.cell_slice(mesh, 2, 5)
    i, jl, k = 1, 2, 1
    assert sl[(i * 3 + jl) * 2 + k] == (i * 7 + 2 + jl) * 2 + k
    sm = sections.sub_mesh(mesh, 2, 5)
    assert sm.shape == (3, 3, 2) and np.array_equal(sm.yn, mesh.yn[2:6])


def test_one_section_without_trends_is_the_plain_inversion():
    p, d_obs, _ = _regional()
    m, m_res, info = sections.invert_sections(p.mesh, p.obs, d_obs, p.wdepth, [0, p.mesh.ny],
                                              data_degree=0, model_degree=0)
    G = np.stack([prism.sensitivity_row(p.mesh, p.obs.x[o], p.obs.y[o], p.obs.z[o])
                  for o in range(p.obs.n)])
    cov = inversion.covariance_from_weights(p.wdepth)
    lam = inversion.lambda_rule(float(np.einsum("ok,k,ok->", G, cov, G)), p.obs.n)
    ref, _ = inversion.invert_dense(G, cov, lam, d_obs)
    np.testing.assert_allclose(m, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert np.array_equal(m, m_res) and abs(info[0]["lam"] - lam) <= 1e-14 * lam


@pytest.mark.parametrize("scope", ["section", "domain"])
def test_each_section_meets_the_model_space_optimality_condition(scope):
    """Eq. 8 at each section's solution: G_s^T (d_s - G_s m_s) / lambda_s =
    C_s^-1 m_s, with d_s the section's trend-removed data."""
    p, d_obs, _ = _regional()
    ysplit = [0, 3, 6, 9]
    m, _, info = sections.invert_sections(p.mesh, p.obs, d_obs, p.wdepth, ysplit, data_degree=2,
                                          data_scope=scope, model_degree=2)
    for s in range(3):
        j0, j1 = ysplit[s], ysplit[s + 1]
        sm = sections.sub_mesh(p.mesh, j0, j1)
        cells = sections.cell_slice(p.mesh, j0, j1)
        so = p.obs.take(info[s]["rows"])
        G = np.stack([prism.sensitivity_row(sm, so.x[o], so.y[o], so.z[o]) for o in range(so.n)])
        ms = m[cells]
        lhs = G.T @ (info[s]["d_in"] - G @ ms) / info[s]["lam"]
        rhs = ms / inversion.covariance_from_weights(p.wdepth[cells])
        assert np.linalg.norm(lhs - rhs) <= 1e-7 * np.linalg.norm(rhs)


def test_regional_field_alone_inverts_to_zero():
    """Data that are exactly a second-degree field: the per-section trend
    removal takes all of it, so every section's model is zero."""
    p, _, regional = _regional()
    m, m_res, _ = sections.invert_sections(p.mesh, p.obs, regional, p.wdepth, [0, 3, 6, 9],
                                           data_degree=2, model_degree=2)
    assert np.abs(m).max() <= 1e-9 * np.abs(regional).max() / prism.GAMMA
    # without the trend removal the same data give a non-zero model
    m0, _, _ = sections.invert_sections(p.mesh, p.obs, regional, p.wdepth, [0, 3, 6, 9],
                                        data_degree=0, model_degree=0)
    assert np.abs(m0).max() > 1e3 * np.abs(m).max()


def test_model_trend_removes_planted_layer_polynomials():
    """Adding a different second-degree polynomial of (x, y) to every layer
    leaves the model residual unchanged; a model that is such a polynomial in
    every layer has zero residual; the residual of a layer is orthogonal to
    the monomials over the cell centres."""
    mesh = workloads.regular_mesh(7, 9, 3, 40.0, 30.0, 20.0, x0=100.0, y0=-50.0)
    rng = np.random.default_rng(8)
    m = rng.standard_normal(mesh.ncells)
    xc = 0.5 * (mesh.xn[:-1] + mesh.xn[1:])
    yc = 0.5 * (mesh.yn[:-1] + mesh.yn[1:])
    X, Y = np.meshgrid(xc, yc, indexing="ij")
    Q = np.stack([c[0] + c[1] * X + c[2] * Y + c[3] * X * X + c[4] * X * Y + c[5] * Y * Y
                  for c in rng.standard_normal((3, 6)) * [1, 1e-2, 1e-2, 1e-4, 1e-4, 1e-4]], axis=2)
    r = sections.model_trend_residual(mesh, m, 2)
    r2 = sections.model_trend_residual(mesh, m + Q.reshape(-1), 2)
    np.testing.assert_allclose(r2, r, atol=1e-9)
    assert np.abs(sections.model_trend_residual(mesh, Q.reshape(-1), 2)).max() <= 1e-9
    B = trend.monomials(X.reshape(-1) - X.mean(), Y.reshape(-1) - Y.mean(), 2)
    for k in range(mesh.nz):
        rk = r.reshape(mesh.shape)[:, :, k].reshape(-1)
        assert np.abs(B.T @ rk).max() <= 1e-8 * np.abs(B).max() * np.abs(rk).sum()
    assert np.array_equal(sections.model_trend_residual(mesh, m, 0), m)
