"""Pins of the FP64 oracle against facts fixed by physics, mathematics and the
paper (not against itself).  CPU only.

Each test states which mistake it would catch: a wrong vertex parity or sign
convention (slab, point mass, reflection), a dropped or mis-indexed term
(superposition, mpmath, index order, point mass), a transposed operand
(adjoint, Eq. 9), a wrong regrouping (literal vs node-shared)."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import GAMMA, prism, inversion, trend
from workloads import Mesh, Survey, random_case, regular_mesh, dykes_32x32x16


def _one_prism(x0, x1, y0, y1, z0, z1):
    return Mesh(np.array([x0, x1]), np.array([y0, y1]), np.array([z0, z1]))


def _gz_single(mesh, xo, yo, zo, rho=1.0):
    obs = Survey(np.array([xo]), np.array([yo]), np.array([zo]))
    return float(prism.forward_literal(mesh, obs, np.array([rho]))[0])


# ---------------------------------------------------------------- Eq. 1-3

def test_bouguer_slab_limit():
    """A square slab of half-width L, thickness h, observed above its centre,
    pulls 2*pi*G*rho*h as L/h -> infinity; the deficit falls like h/L and is
    positive (the slab pulls down, z down => gz > 0)."""
    h, rho, height = 10.0, 1000.0, 5.0
    target = 2 * math.pi * GAMMA * rho * h
    ratios = []
    for L in [1e2, 1e3, 1e4, 1e5, 1e7]:
        mesh = _one_prism(-L, L, -L, L, 0.0, h)
        ratios.append(_gz_single(mesh, 0.0, 0.0, -height, rho) / target)
    ratios = np.array(ratios)
    assert np.all(np.diff(ratios) > 0), ratios           # monotone convergence
    assert np.all(ratios < 1.0)
    assert abs(ratios[2] - 1) < 1e-3                      # L/h = 1e3
    assert abs(ratios[3] - 1) < 2e-4                      # L/h = 1e4
    assert abs(ratios[4] - 1) < 5e-6                      # L/h = 1e6
    # Far-field deficit: the part of the infinite slab outside the square,
    # int_{outside} zbar/r^3 dA = zbar * 4*sqrt(2)/L, so
    # (1 - ratio) * L / zbar -> 2*sqrt(2)/pi, zbar = mean depth of the slab.
    zbar = height + h / 2
    defic = (1 - ratios[1:4]) * np.array([1e3, 1e4, 1e5]) / zbar
    np.testing.assert_allclose(defic[1:], 2 * math.sqrt(2) / math.pi, rtol=1e-4)


def test_cube_far_field_is_point_mass():
    """Far from a cube its field is that of a point mass gamma*rho*a^3 at the
    centre: gz = gamma*M*(z_c - z_o)/R^3, with relative error O((a/R)^4)
    (a cube has no quadrupole)."""
    a, rho = 10.0, 2500.0
    c = np.array([3.0, -7.0, 500.0])
    mesh = _one_prism(c[0] - a / 2, c[0] + a / 2, c[1] - a / 2, c[1] + a / 2,
                      c[2] - a / 2, c[2] + a / 2)
    rng = np.random.default_rng(11)
    for _ in range(4):
        d = rng.standard_normal(3)
        d[2] = -abs(d[2]) - 0.2          # observation above the cube
        d /= np.linalg.norm(d)
        o = c + 100 * a * d
        gz = _gz_single(mesh, *o, rho=rho)
        R = np.linalg.norm(c - o)
        pm = GAMMA * rho * a ** 3 * (c[2] - o[2]) / R ** 3
        assert gz > 0
        assert abs(gz - pm) / abs(pm) < 1e-6


def test_elongated_prism_far_field_quadrupole_scaling():
    """A non-cubic prism differs from the point mass by O((a/R)^2): the error
    drops ~100x per 10x distance (a missing/extra term would not)."""
    c = np.array([0.0, 0.0, 800.0])
    half = np.array([40.0, 10.0, 5.0])
    mesh = _one_prism(*(c[0] + np.array([-1, 1]) * half[0]), *(c[1] + np.array([-1, 1]) * half[1]),
                      *(c[2] + np.array([-1, 1]) * half[2]))
    d = np.array([0.3, 0.5, -0.81])
    d /= np.linalg.norm(d)
    errs = []
    for R in [1e3, 1e4]:   # far enough for the quadrupole, near enough for FP64
        o = c + R * d
        gz = _gz_single(mesh, *o)
        mass = np.prod(2 * half)
        pm = GAMMA * mass * (c[2] - o[2]) / R ** 3
        errs.append(abs(gz - pm) / abs(pm))
    assert 70 < errs[0] / errs[1] < 140, errs


def test_voxel_sphere_converges_to_analytic_sphere():
    """A sphere assembled from cubic cells: outside it, gz equals the point
    mass of the voxelised mass; the multipole error shrinks with refinement."""
    r, rho = 100.0, 500.0
    centre = np.array([0.0, 0.0, 300.0])
    obs = Survey(np.array([0.0, 150.0, -220.0]), np.array([0.0, 60.0, 90.0]),
                 np.array([-10.0, 0.0, -50.0]))
    errs_pm, errs_an = [], []
    for n in (10, 20, 40):
        a = 2 * r / n
        nodes = np.arange(n + 1) * a - r
        mesh = Mesh(nodes + centre[0], nodes + centre[1], nodes + centre[2])
        X, Y, Z = np.meshgrid(*(0.5 * (v[1:] + v[:-1]) for v in (mesh.xn, mesh.yn, mesh.zn)),
                              indexing="ij")
        inside = ((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2) <= r * r
        m = rho * inside.reshape(-1).astype(float)
        gz = prism.forward(mesh, obs, m)
        mass = m.sum() * a ** 3
        R = np.sqrt((centre[0] - obs.x) ** 2 + (centre[1] - obs.y) ** 2 + (centre[2] - obs.z) ** 2)
        ref = GAMMA * mass * (centre[2] - obs.z) / R ** 3
        analytic = GAMMA * rho * (4 / 3) * math.pi * r ** 3 * (centre[2] - obs.z) / R ** 3
        errs_pm.append(np.max(np.abs(gz - ref) / np.abs(ref)))
        errs_an.append(np.max(np.abs(gz - analytic) / analytic))
    # the voxel body (cubic symmetry, no quadrupole) acts as its own mass at the centre
    assert max(errs_pm) < 2e-4 and errs_pm[2] < 2e-5, errs_pm
    # and converges to the analytic sphere as the voxelisation is refined
    assert errs_an[0] > errs_an[1] > errs_an[2], errs_an
    assert errs_an[2] < 2e-3


def test_superposition_of_sub_prisms():
    """One prism equals the sum of its 2x3x4 sub-prisms (Eq. 4)."""
    big = _one_prism(-20.0, 35.0, 10.0, 50.0, 5.0, 65.0)
    sub = Mesh(np.array([-20.0, 3.7, 35.0]), np.array([10.0, 17.0, 31.5, 50.0]),
               np.array([5.0, 9.0, 30.0, 41.0, 65.0]))
    rng = np.random.default_rng(3)
    obs = Survey(rng.uniform(-100, 100, 12), rng.uniform(-60, 120, 12), rng.uniform(-30, 5, 12))
    one = prism.forward_literal(big, obs, np.array([700.0]))
    many = prism.forward_literal(sub, obs, np.full(sub.ncells, 700.0))
    np.testing.assert_allclose(many, one, rtol=1e-12, atol=0)


def test_mirror_symmetry_x_and_y():
    """Mirroring mesh, model and observations in x (or y) leaves gz unchanged."""
    p = random_case(5, 4, 5, 3, 9, rectilinear=True)
    mesh, obs, m = p.mesh, p.obs, p.m
    d = prism.forward(mesh, obs, m)
    mx = Mesh(-mesh.xn[::-1], mesh.yn, mesh.zn)
    m_x = m.reshape(mesh.shape)[::-1, :, :].reshape(-1)
    d_x = prism.forward(mx, Survey(-obs.x, obs.y, obs.z), m_x)
    my = Mesh(mesh.xn, -mesh.yn[::-1], mesh.zn)
    m_y = m.reshape(mesh.shape)[:, ::-1, :].reshape(-1)
    d_y = prism.forward(my, Survey(obs.x, -obs.y, obs.z), m_y)
    scale = np.max(np.abs(d))
    assert np.max(np.abs(d_x - d)) < 1e-12 * scale
    assert np.max(np.abs(d_y - d)) < 1e-12 * scale


def test_reflection_through_mid_depth_flips_sign():
    """An observation reflected through the mid-depth plane of an isolated
    prism sees the opposite vertical attraction (oracle only: the library
    rejects observations below the mesh top)."""
    mesh = _one_prism(0.0, 10.0, 0.0, 20.0, 100.0, 150.0)
    for (xo, yo, dz) in [(3.0, 4.0, 30.0), (-50.0, 70.0, 5.0), (5.0, 10.0, 200.0)]:
        above = _gz_single(mesh, xo, yo, 100.0 - dz)
        below = _gz_single(mesh, xo, yo, 150.0 + dz)
        assert above > 0
        assert abs(above + below) <= 1e-12 * abs(above)


def _psi_mp(x, y, z):
    x, y, z = mp.mpf(x), mp.mpf(y), mp.mpf(z)
    R = mp.sqrt(x * x + y * y + z * z)
    t = z * mp.atan(x * y / (z * R)) if z != 0 else mp.mpf(0)
    lx = x * mp.log(R + y) if x != 0 else mp.mpf(0)
    ly = y * mp.log(R + x) if y != 0 else mp.mpf(0)
    return t - lx - ly


def _corner_sum_mp(x1, x2, y1, y2, z1, z2):
    xs, ys, zs = (x1, x2), (y1, y2), (z1, z2)
    s = mp.mpf(0)
    for p in (1, 2):
        for q in (1, 2):
            for r in (1, 2):
                s += (-1) ** (p + q + r) * _psi_mp(xs[p - 1], ys[q - 1], zs[r - 1])
    return s


@pytest.mark.parametrize("ratio", [1, 10, 100, 1000])
def test_prism_against_50_digit_literal_formula(ratio):
    """Per-prism corner sum (Eq. 1-3, evaluated literally with plain ln(R+y)
    in 50-digit arithmetic) vs the FP64 oracle, whose error may grow like
    eps*(R/a)^3*ln(R) from the cancellation between corners."""
    mp.mp.dps = 50
    a = 10.0
    rng = np.random.default_rng(100 + ratio)
    c = np.array([1.0, -2.0, 200.0])
    for _ in range(3):
        d = rng.standard_normal(3)
        d[2] = -abs(d[2]) - 0.3
        d /= np.linalg.norm(d)
        R = ratio * a
        o = c + R * d
        args = (c[0] - a / 2 - o[0], c[0] + a / 2 - o[0], c[1] - a / 2 - o[1],
                c[1] + a / 2 - o[1], c[2] - a / 2 - o[2], c[2] + a / 2 - o[2])
        f = prism.prism_corner_sum(*args)
        e = _corner_sum_mp(*args)
        rel = abs((mp.mpf(float(f)) - e) / e)
        tol = 20 * 1.1e-16 * max(1.0, ratio) ** 3 * max(1.0, math.log(R))
        assert float(rel) < tol, (ratio, float(rel), tol)


def test_psi_rationalised_logs_near_singular_line():
    """ln(R+y) for y << 0 with x, z small: the oracle's rationalised form keeps
    full precision where the literal R+y would cancel (50-digit reference)."""
    mp.mp.dps = 50
    for (x, y, z) in [(25.0, -5000.0, 25.0), (-0.5, -800.0, 3.0), (1e-3, -1e4, 2.0),
                      (-3000.0, 2.0, 1.0)]:
        ref = _psi_mp(x, y, z)
        got = prism.psi(x, y, z)
        assert abs((mp.mpf(float(got)) - ref) / ref) < 1e-14


def test_psi_singular_limits():
    """The select-based limits equal the continuous limits of Eq. 2."""
    assert prism.psi(0.0, 0.0, 0.0) == 0.0
    for (y, z) in [(3.0, 4.0), (-3.0, 4.0), (5.0, 0.0), (-5.0, 0.0)]:
        assert abs(prism.psi(1e-12, y, z) - prism.psi(0.0, y, z)) < 1e-9
        assert abs(prism.psi(y, 1e-12, z) - prism.psi(y, 0.0, z)) < 1e-9
    for (x, y) in [(3.0, 4.0), (-3.0, 4.0), (2.0, -7.0)]:
        assert abs(prism.psi(x, y, 1e-12) - prism.psi(x, y, 0.0)) < 1e-9


# ---------------------------------------------------------------- Eq. 4-6

def test_node_shared_equals_literal():
    """The node-shared regrouping equals the literal per-prism sum, for the
    forward, the adjoint, rows of G and the weighted row sums; including
    observations on nodes and on the mesh top."""
    p = random_case(7, 3, 4, 5, 11, on_nodes=3, on_top=4)
    G = prism.sensitivity_literal(p.mesh, p.obs)
    d = prism.forward(p.mesh, p.obs, p.m)
    np.testing.assert_allclose(d, G @ p.m, rtol=1e-11, atol=1e-12 * np.abs(G @ p.m).max())
    g = prism.adjoint(p.mesh, p.obs, p.probe_v)
    ref = G.T @ p.probe_v
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-11 * np.abs(ref).max())
    cells = np.array([0, 5, 17, p.mesh.ncells - 1])
    np.testing.assert_allclose(prism.adjoint_cells(p.mesh, p.obs, p.probe_v, cells), ref[cells],
                               rtol=1e-10, atol=1e-11 * np.abs(ref).max())
    for o in (0, 6, 10):
        row = prism.sensitivity_row(p.mesh, p.obs.x[o], p.obs.y[o], p.obs.z[o])
        np.testing.assert_allclose(row, G[o], rtol=1e-10, atol=1e-12 * np.abs(G[o]).max())
    cov = inversion.covariance_from_weights(p.wdepth)
    np.testing.assert_allclose(prism.weighted_row_sumsq(p.mesh, p.obs, cov),
                               np.einsum("ok,k,ok->o", G, cov, G), rtol=1e-10)
    models = np.stack([p.m, -2 * p.m + 1.0], axis=1)
    np.testing.assert_allclose(prism.forward_multi(p.mesh, p.obs, models), G @ models,
                               rtol=1e-10, atol=1e-12 * np.abs(G @ models).max())


def test_single_cell_index_order():
    """Flat index (i*ny + j)*nz + k (z fastest): a single non-zero cell gives
    exactly that prism's field."""
    mesh = regular_mesh(4, 3, 5, 10.0, 20.0, 7.0, x0=-15.0)
    obs = Survey(np.array([3.0, -40.0]), np.array([11.0, 70.0]), np.array([-1.0, 0.0]))
    i, j, k = 2, 1, 3
    m = np.zeros(mesh.ncells)
    m[(i * mesh.ny + j) * mesh.nz + k] = 1.0
    one = _one_prism(mesh.xn[i], mesh.xn[i + 1], mesh.yn[j], mesh.yn[j + 1], mesh.zn[k], mesh.zn[k + 1])
    np.testing.assert_allclose(prism.forward(mesh, obs, m), prism.forward_literal(one, obs, [1.0]),
                               rtol=1e-12)


def test_constant_block_node_weights_only_at_corners():
    """For a constant-density block the node weights vanish except at the
    block's 8 corners, where they carry +-rho with the vertex parity."""
    mesh = regular_mesh(6, 5, 4, 1.0, 1.0, 1.0)
    m = np.zeros(mesh.shape)
    m[1:4, 2:5, 1:3] = 2.0
    W = prism.node_weights(mesh, m.reshape(-1))
    nz_idx = np.argwhere(W != 0)
    assert len(nz_idx) == 8
    for (a, b, c) in nz_idx:
        p = 1 if a == 1 else 2
        q = 1 if b == 2 else 2
        r = 1 if c == 1 else 2
        assert W[a, b, c] == (-1.0) ** (p + q + r) * 2.0


# ---------------------------------------------------------------- Eq. 7-11

def _tiny_problem(seed=3):
    p = random_case(seed, 4, 4, 3, 10, model="blocky")
    G = prism.sensitivity_literal(p.mesh, p.obs)
    cov = inversion.covariance_from_weights(p.wdepth)
    d_clean = G @ p.m
    d_obs = inversion.add_noise(d_clean, p.noise_draws, 0.01)
    tr = float(np.einsum("ok,k,ok->", G, cov, G))
    lam = inversion.lambda_rule(tr, p.obs.n)
    return p, G, cov, d_obs, lam


def test_adjoint_dot_product():
    """<G m, v> = <m, G^T v> for the matrix-free operators."""
    p = random_case(9, 5, 4, 6, 13)
    lhs = np.dot(prism.forward(p.mesh, p.obs, p.m), p.probe_v)
    rhs = np.dot(p.m, prism.adjoint(p.mesh, p.obs, p.probe_v))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_dataspace_apply_matches_dense():
    p, G, cov, d_obs, lam = _tiny_problem()
    v = p.probe_v
    A = inversion.dataspace_matrix(G, cov, lam)
    got = inversion.dataspace_apply(p.mesh, p.obs, p.wdepth, lam, v)
    np.testing.assert_allclose(got, A @ v, rtol=1e-10, atol=1e-12 * np.abs(A @ v).max())


def test_eq9_identity_model_space_equals_data_space():
    """Eq. 8 solved in model space equals Eq. 11 solved in data space."""
    p, G, cov, d_obs, lam = _tiny_problem()
    m_ref = np.full(p.mesh.ncells, 0.1)
    m_data, _ = inversion.invert_dense(G, cov, lam, d_obs, m_ref)
    m_model = inversion.invert_model_space(G, cov, lam, d_obs, m_ref)
    np.testing.assert_allclose(m_data, m_model, rtol=1e-9, atol=1e-10 * np.abs(m_model).max())


def test_solution_is_stationary_point_of_objective():
    """The data-space solution zeroes the gradient of phi (Eq. 7):
    -G^T W_d^-1 (d - G m) + W_m^-1 (m - m_ref) = 0."""
    p, G, cov, d_obs, lam = _tiny_problem(4)
    m_ref = np.zeros(p.mesh.ncells)
    m, _ = inversion.invert_dense(G, cov, lam, d_obs, m_ref)
    t1 = -G.T @ (d_obs - G @ m) / lam
    t2 = (m - m_ref) / cov
    assert np.linalg.norm(t1 + t2) <= 1e-8 * np.linalg.norm(t2)


def test_cg_converges_to_cholesky():
    p, G, cov, d_obs, lam = _tiny_problem(5)
    m_chol, y_chol = inversion.invert_dense(G, cov, lam, d_obs)
    m_cg, y_cg, it, hist = inversion.invert_cg(p.mesh, p.obs, d_obs, p.wdepth, lam, tol=1e-13,
                                               max_iter=200)
    assert hist[-1] <= 1e-13
    assert np.linalg.norm(m_cg - m_chol) <= 1e-9 * np.linalg.norm(m_chol)
    assert np.linalg.norm(y_cg - y_chol) <= 1e-9 * np.linalg.norm(y_chol)


def test_cg_fixed_iterations_and_history():
    p, G, cov, d_obs, lam = _tiny_problem(6)
    A = inversion.dataspace_matrix(G, cov, lam)
    y, it, hist = inversion.conjugate_gradient(lambda v: A @ v, d_obs, fixed_iters=4)
    assert it == 4 and len(hist) == 5
    assert np.isclose(hist[-1], np.linalg.norm(d_obs - A @ y) / np.linalg.norm(d_obs), rtol=1e-6)


def test_noise_model_relative_rms_and_r2_scaling():
    """Noise = level * RMS(d) * N(0,1) draws.  With d_calc ~ d_clean,
    1 - R^2 ~ level^2 RMS^2 / var(d), so it grows ~4x from 1 % to 2 %; the
    paper's pair of values (4e-4 -> 1.4e-3) has the same ~3.5-4x ratio (weak,
    consistency-only check)."""
    d = np.sin(np.linspace(0, 9, 4000)) + 2.0
    draws = np.random.default_rng(0).standard_normal(d.size)
    n1 = inversion.add_noise(d, draws, 0.01) - d
    n2 = inversion.add_noise(d, draws, 0.02) - d
    rms = np.sqrt(np.mean(d * d))
    assert abs(np.sqrt(np.mean(n1 ** 2)) / rms - 0.01) < 0.001

    def one_minus_r2(dobs):
        return np.sum((dobs - d) ** 2) / np.sum((dobs - dobs.mean()) ** 2)
    ratio = one_minus_r2(d + n2) / one_minus_r2(d + n1)
    assert 3.0 < ratio < 5.0
    assert 3.0 < (1 - 0.9986) / (1 - 0.9996) < 4.0


def test_dykes_32x32x16_model_geometry():
    """Input recipe check: both dykes are 2 cells wide, 8 long, 10 deep."""
    p = dykes_32x32x16()
    assert p.mesh.ncells == 16384 and p.obs.n == 1024
    assert int((p.m > 0).sum()) == 320
    assert np.all(p.obs.z == p.mesh.zn[0])


def test_restarted_cg_policy_converges_to_cholesky():
    """The restarted policy reaches the Cholesky solution of Eq. 11 given
    enough cycles (short cycles: 4 inner iterations), and the quadratic it
    minimises, Q(y) = y^T A y / 2 - y^T b, never rises from one cycle to the next."""
    p, G, cov, d_obs, lam = _tiny_problem(8)
    A = inversion.dataspace_matrix(G, cov, lam)
    y_chol = np.linalg.solve(A, d_obs)
    y, total, cycles, hist = inversion.restarted_cg(lambda v: A @ v, d_obs, inner=4, outer=200,
                                                    tol=1e-12)
    assert hist[-1] <= 1e-12 and cycles < 200 and total <= 4 * cycles
    assert np.linalg.norm(y - y_chol) <= 1e-9 * np.linalg.norm(y_chol)
    qs = []
    for k in range(1, 8):
        yk, _, _, _ = inversion.restarted_cg(lambda v: A @ v, d_obs, inner=2, outer=k, tol=0.0)
        qs.append(0.5 * yk @ A @ yk - yk @ d_obs)
    assert np.all(np.diff(qs) <= 1e-12 * abs(qs[0]))
    # one long cycle is plain CG: 20 inner iterations on N = 10 reach the solution
    y1, total1, cycles1, _ = inversion.restarted_cg(lambda v: A @ v, d_obs, tol=1e-12)
    y_cg, it_cg, _ = inversion.conjugate_gradient(lambda v: A @ v, d_obs, tol=1e-12, max_iter=20)
    assert cycles1 == 1 and total1 == it_cg
    np.testing.assert_allclose(y1, y_cg, rtol=1e-12, atol=1e-12 * np.abs(y_cg).max())


def test_restarted_cg_backtracking_halves_a_rising_step():
    """Backtracking: with an operator whose cycle overshoots (a large skew part
    makes CG steps too long for the symmetric quadratic), the unguarded cycle
    raises Q above Q(0) = 0 and the guarded one halves the step back below it."""
    rng = np.random.default_rng(0)
    n = 12
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    S = Q @ np.diag(np.logspace(0, 3, n)) @ Q.T
    K = rng.standard_normal((n, n))
    A = S + 50.0 * (K - K.T)
    b = rng.standard_normal(n)
    quad = lambda y: 0.5 * y @ S @ y - y @ b  # noqa: E731  (y^T A y = y^T S y)
    y0, _, _, _ = inversion.restarted_cg(lambda v: A @ v, b, inner=5, outer=1, tol=0.0,
                                         max_halvings=0)
    y1, _, _, _ = inversion.restarted_cg(lambda v: A @ v, b, inner=5, outer=1, tol=0.0)
    assert quad(y0) > 0.0 > quad(y1)
    # the guarded step is the unguarded one halved k times
    ratios = y1 / y0
    assert np.allclose(ratios, ratios[0]) and np.log2(1.0 / ratios[0]) in (1, 2, 3, 4, 5)


# ------------------------------------------------------------------ trend surface

def _stations(seed, n):
    rng = np.random.default_rng(seed)
    return rng.uniform(2.0e5, 3.3e5, n), rng.uniform(2.6e6, 2.82e6, n), rng


def test_trend_surface_recovers_planted_quadratic():
    """A field that is exactly a second-degree polynomial is its own trend:
    residual zero to rounding; a first-degree fit of a plane likewise."""
    x, y, rng = _stations(1, 500)
    u, w = (x - 2.6e5) / 1e5, (y - 2.7e6) / 1e5
    quad = 3.0 - 1.5 * u + 0.7 * w + 0.25 * u * u - 0.4 * u * w + 0.9 * w * w
    t, r = trend.trend_surface(x, y, quad, 2)
    assert np.abs(r).max() <= 1e-10 * np.abs(quad).max()
    plane = 3.0 - 1.5 * u + 0.7 * w
    t1, r1 = trend.trend_surface(x, y, plane, 1)
    assert np.abs(r1).max() <= 1e-10 * np.abs(plane).max()


def test_trend_surface_residual_is_orthogonal_to_the_basis():
    """Normal equations: the residual is orthogonal to every monomial of the
    degree, and adding any such polynomial to the data leaves it unchanged."""
    x, y, rng = _stations(2, 700)
    v = rng.standard_normal(700) + np.sin(x / 2e4)
    _, r = trend.trend_surface(x, y, v, 2)
    xs, ys = (x - x.min()) / 1e5, (y - y.min()) / 1e5
    for col in (np.ones_like(xs), xs, ys, xs * xs, xs * ys, ys * ys):
        assert abs(col @ r) <= 1e-10 * np.linalg.norm(col) * np.linalg.norm(v)
    _, r2 = trend.trend_surface(x, y, v + 5.0 + 2.0 * xs - 3.0 * xs * ys, 2)
    np.testing.assert_allclose(r2, r, atol=1e-10 * np.abs(v).max())


def test_trend_surface_plane_on_symmetric_grid_closed_form():
    """On a grid symmetric about its centre the monomials 1, u, w are
    orthogonal, so the first-degree fit is mean(v) + u S_uv / S_uu + w S_wv / S_ww."""
    u, w = np.meshgrid(np.linspace(-3, 3, 13), np.linspace(-2, 2, 9), indexing="ij")
    u, w = u.ravel(), w.ravel()
    v = np.random.default_rng(4).standard_normal(u.size) + np.cos(u * w)
    t, _ = trend.trend_surface(1e3 * u + 4e5, 1e3 * w + 7e6, v, 1)
    closed = v.mean() + u * (u @ v) / (u @ u) + w * (w @ v) / (w @ w)
    np.testing.assert_allclose(t, closed, atol=1e-12 * np.abs(v).max())


def test_cg_warm_start_resumes_the_solve():
    """Warm start: starting from the exact solution stops at once; resuming a
    stopped solve from its iterate reaches the Cholesky solution; the history
    starts at the relative residual of the starting iterate."""
    p, G, cov, d_obs, lam = _tiny_problem(9)
    A = inversion.dataspace_matrix(G, cov, lam)
    y_chol = np.linalg.solve(A, d_obs)
    y, it, hist = inversion.conjugate_gradient(lambda v: A @ v, d_obs, tol=1e-10, y0=y_chol)
    assert it == 0 and hist[0] <= 1e-10
    y4, _, _ = inversion.conjugate_gradient(lambda v: A @ v, d_obs, fixed_iters=4)
    y_res, it_res, h_res = inversion.conjugate_gradient(lambda v: A @ v, d_obs, tol=1e-12,
                                                        max_iter=100, y0=y4)
    assert np.isclose(h_res[0], np.linalg.norm(d_obs - A @ y4) / np.linalg.norm(d_obs), rtol=1e-12)
    assert np.linalg.norm(y_res - y_chol) <= 1e-9 * np.linalg.norm(y_chol)
    y_r, _, cycles, _ = inversion.restarted_cg(lambda v: A @ v, d_obs, inner=20, outer=30,
                                               tol=1e-12, y0=y4)
    assert np.linalg.norm(y_r - y_chol) <= 1e-9 * np.linalg.norm(y_chol)
    _, tot0, cyc0, _ = inversion.restarted_cg(lambda v: A @ v, d_obs, tol=1e-8, y0=y_chol)
    assert tot0 == 0 and cyc0 == 0
