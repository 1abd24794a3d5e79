"""Bounds that the deep-layer edge formula of the GPU sweeps relies on.

In a layer whose top lies at least 9 thicknesses below the mesh top, every
observation on or above the top sees z1 >= 9 h.  The deep-layer formula then
(a) evaluates the atan of the difference term z1 atan(u1) -> atan(delta) with
a short odd polynomial that is accurate for |delta| <= 1/8, and (b) adds the
rounding error of 1 + t in log1p(t) without the 1/u factor, which is accurate
for t < 1/4.  Both bounds are facts about the edge-segment formula (Eq. 1-3
written as a difference over one vertical edge); this test samples them in
FP64, including the worst cases (observation close to the column, one of x, y
zero or negative, z1 at its smallest)."""
import numpy as np

DEEP_RATIO = 9.0


def _terms(x, y, z1, h):
    z2 = z1 + h
    s = x * x + y * y
    r1 = np.sqrt(s + z1 * z1)
    r2 = np.sqrt(s + z2 * z2)
    dr = h * (z1 + z2) / (r1 + r2)
    # 1/(R1 + y) without cancellation: rationalised for y < 0
    inv_y = np.where(y >= 0, 1.0 / (r1 + np.abs(y)), (r1 + np.abs(y)) / (x * x + z1 * z1))
    inv_x = np.where(x >= 0, 1.0 / (r1 + np.abs(x)), (r1 + np.abs(x)) / (y * y + z1 * z1))
    u1 = x * y / (z1 * r1)
    u2 = x * y / (z2 * r2)
    delta = (u2 - u1) / (1.0 + u1 * u2)
    return dr * inv_y, dr * inv_x, delta


def _samples(rng, n):
    h = rng.uniform(1.0, 300.0, n)
    z1 = h * (DEEP_RATIO + rng.exponential(3.0, n) * (rng.random(n) < 0.7))
    scale = z1 * 10.0 ** rng.uniform(-3, 3, n)
    x = rng.standard_normal(n) * scale
    y = rng.standard_normal(n) * scale
    # one offset zero, or both, in a share of the samples
    x[rng.random(n) < 0.1] = 0.0
    y[rng.random(n) < 0.1] = 0.0
    return x, y, z1, h


def test_log1p_arguments_below_a_quarter_in_deep_layers():
    rng = np.random.default_rng(11)
    x, y, z1, h = _samples(rng, 400_000)
    ty, tx = _terms(x, y, z1, h)[:2]
    bound = 2.0 / DEEP_RATIO + 1.0 / DEEP_RATIO ** 2
    assert np.all(ty >= 0) and np.all(tx >= 0)
    assert ty.max() <= bound * (1 + 1e-12) and tx.max() <= bound * (1 + 1e-12)
    assert bound < 0.25
    # the bound is approached: observation far along -y, x = 0, z1 = 9 h
    hh = np.array([50.0])
    t_edge = _terms(np.array([0.0]), np.array([-1e9]), DEEP_RATIO * hh, hh)[0][0]
    assert t_edge > 0.99 * bound


def test_atan_difference_below_an_eighth_in_deep_layers():
    rng = np.random.default_rng(12)
    x, y, z1, h = _samples(rng, 400_000)
    delta = _terms(x, y, z1, h)[2]
    assert np.abs(delta).max() <= 10.0 / 81.0 * (1 + 1e-12)
    assert 10.0 / 81.0 < 0.125


def test_bounds_fail_above_the_deep_threshold():
    # at z1 = 2 h the log1p argument can exceed 1/4: the threshold matters
    h = np.array([100.0])
    t = _terms(np.array([0.0]), np.array([-1e9]), 2.0 * h, h)[0][0]
    assert t > 0.25


def test_log1p_without_the_inverse_factor():
    # u = fl32(1 + t), c = t - (u - 1) exact; ln(u) + c against log1p(t), with
    # ln(u) taken exact so that only the dropped factor 1/u is measured.  The
    # difference |c| (u - 1) / u is at most 2^-24 (t + 2^-24) < 2^-23 t (worst
    # just above t = 2^-24, where u rounds up to 1 + 2^-23), and about
    # 2^-24 t once t >> 2^-24.
    rng = np.random.default_rng(13)
    t = np.concatenate([rng.uniform(0.0, 0.25, 200_000),
                        10.0 ** rng.uniform(-9, np.log10(0.25), 200_000)]).astype(np.float32)
    u = (np.float32(1.0) + t).astype(np.float32)
    c = (t - (u - np.float32(1.0))).astype(np.float32)
    t64, u64, c64 = t.astype(np.float64), u.astype(np.float64), c.astype(np.float64)
    assert np.array_equal(u64 + c64, 1.0 + t64)          # c is the exact rounding error
    approx = np.log(u64) + c64
    exact = np.log1p(t64)
    ok = exact > 0
    rel = np.abs(approx[ok] - exact[ok]) / exact[ok]
    assert rel.max() <= 1.2e-7
    big = t64[ok] > 2.0 ** -16
    assert rel[big].max() <= 1.01 * 2.0 ** -24
    # near the worst case, t just above 2^-24, the error exceeds 2^-24 t
    # (0.75 * 2^-23 t: the -t^2/2 of log1p cancels a quarter of it)
    tw = np.float32(2.0 ** -24 * (1 + 2.0 ** -20))
    uw = np.float32(np.float32(1.0) + tw)
    cw = np.float64(np.float32(tw - (uw - np.float32(1.0))))
    rw = abs(np.log(np.float64(uw)) + cw - np.log1p(np.float64(tw))) / np.log1p(np.float64(tw))
    assert 1.4 * 2.0 ** -24 < rw < 2.0 ** -23


def _column_walk(rng, n, layers):
    """n columns, each walked down `layers` deep layers: offsets (x, y) and node
    depths z_0 < ... < z_layers with z_0 >= 9 h_0 and thicknesses growing
    downwards, as in the benchmark meshes."""
    h0 = rng.uniform(1.0, 300.0, n)
    z0 = h0 * (DEEP_RATIO + rng.exponential(3.0, n) * (rng.random(n) < 0.7))
    grow = rng.uniform(1.0, 1.05, n)
    hs = h0[:, None] * grow[:, None] ** np.arange(layers)[None, :]
    z = np.concatenate([z0[:, None], z0[:, None] + np.cumsum(hs, axis=1)], axis=1)
    scale = z0 * 10.0 ** rng.uniform(-3, 3, n)
    x = rng.standard_normal(n) * scale
    y = rng.standard_normal(n) * scale
    x[rng.random(n) < 0.1] = 0.0
    y[rng.random(n) < 0.1] = 0.0
    return x, y, z


def test_atan_addition_formula_down_a_column():
    # atan(u_k) = atan(u_0) + sum_j atan(delta_j) along a column, delta_j the
    # atan-difference argument of segment j: u_j u_{j+1} >= 0, so no branch of
    # atan is crossed, and all delta_j of a column share one sign (u is monotone
    # in z), so their atan terms add up to |atan(u_k) - atan(u_0)| <= pi/2.
    rng = np.random.default_rng(14)
    x, y, z = _column_walk(rng, 50_000, 147)
    s = (x * x + y * y)[:, None]
    r = np.sqrt(s + z * z)
    u = (x * y)[:, None] / (z * r)
    u1, u2 = u[:, :-1], u[:, 1:]
    assert np.all(u1 * u2 >= 0)
    delta = np.arctan((u2 - u1) / (1.0 + u1 * u2))
    walked = np.arctan(u[:, :1]) + np.cumsum(delta, axis=1)
    assert np.abs(walked - np.arctan(u2)).max() <= 1e-13
    same_sign = (np.all(delta <= 0, axis=1) | np.all(delta >= 0, axis=1))
    assert np.all(same_sign)
    assert np.abs(delta).sum(axis=1).max() <= np.pi / 2 * (1 + 1e-12)
    # the closed form of delta used by the sweeps (no difference of u's)
    z1, z2 = z[:, :-1], z[:, 1:]
    hz = (z2 - z1) * (z1 + z2)
    num = -(x * y)[:, None] * hz * (s + z1 * z1 + z2 * z2)
    den = (z1 * r[:, :-1] + z2 * r[:, 1:]) * (z1 * r[:, :-1] * z2 * r[:, 1:] + ((x * y) ** 2)[:, None])
    closed = np.arctan(num / den)
    assert np.abs(closed - delta).max() <= 1e-14


def test_fp32_carried_angle_error_in_sixteen_layer_walks():
    # The adjoint carries the angle in FP32 over walks of at most 16 layers:
    # A_{j+1} = fl32(A_j + fl32(atan(delta_j))).  With correctly rounded terms the
    # error of A after j steps is at most sum of the half-ulp roundings,
    # 2^-24 (|A_0| + sum_i |A_{i+1}| + sum_i |atan(delta_i)|).
    rng = np.random.default_rng(15)
    x, y, z = _column_walk(rng, 100_000, 16)
    r = np.sqrt((x * x + y * y)[:, None] + z * z)
    exact = np.arctan((x * y)[:, None] / (z * r))
    a = exact[:, 0].astype(np.float32)
    bound = 2.0 ** -24 * np.abs(exact[:, 0])
    worst = 0.0
    for j in range(16):
        d = (exact[:, j + 1] - exact[:, j]).astype(np.float32)
        a = (a + d).astype(np.float32)
        bound = bound + 2.0 ** -24 * (np.abs(exact[:, j + 1]) + np.abs(exact[:, j + 1] - exact[:, j]))
        err = np.abs(a.astype(np.float64) - exact[:, j + 1])
        assert np.all(err <= bound * (1 + 1e-6) + 1e-30)
        worst = max(worst, float((err / np.maximum(np.abs(exact[:, 0]), 1e-30)).max()))
    # relative to the walk's largest angle (its first: |u| falls with depth)
    # that is at most 33 roundings; in practice a few
    assert worst < 33 * 2.0 ** -24
