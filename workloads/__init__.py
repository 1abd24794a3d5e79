"""Seeded synthetic inputs for the prism-gravity operators.

This module only *builds inputs*: rectilinear prism meshes (node coordinate
vectors), observation points, density-contrast models, depth-weight vectors
and the random draws used for data noise and probe vectors.  It contains none
of the gravity arithmetic (no Psi, no corner sums, no sensitivities), so the
FP64 CPU oracle and the GPU library can both be fed from it without sharing
any of the method's code.

Conventions (shared by every consumer):

* z points down; ``zn[0]`` is the mesh top; an observation at height ``h``
  above the top has ``z = zn[0] - h``.
* Cell ``(i, j, k)`` spans ``[xn[i], xn[i+1]] x [yn[j], yn[j+1]] x
  [zn[k], zn[k+1]]``; flat density index ``(i * ny + j) * nz + k`` (C order,
  z fastest).  Densities are density contrasts in kg/m^3, lengths in metres.

The five named workloads follow the problem shapes of the paper's experiments
(regular prism meshes, gridded or scattered ground/airborne observations,
dyke- and body-shaped density contrasts, 0-2 % Gaussian data noise; paper
Sections 2-4 and Tables 1-3); the concrete geometry, which the paper does not
publish, is fixed here with explicit seeds.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Mesh", "Survey", "Problem", "regular_mesh", "cell_centres",
    "dykes_32x32x16", "ellipsoids_100x100x50", "smoothed_box_models", "paper_scale", "serving_stream",
    "random_case", "ellipsoid_model", "dyke_model", "regional_sections", "regional_field",
]


@dataclass
class Mesh:
    """Rectilinear prism mesh given by its node coordinate vectors (float64)."""
    xn: np.ndarray
    yn: np.ndarray
    zn: np.ndarray

    def __post_init__(self):
        self.xn = np.ascontiguousarray(self.xn, dtype=np.float64)
        self.yn = np.ascontiguousarray(self.yn, dtype=np.float64)
        self.zn = np.ascontiguousarray(self.zn, dtype=np.float64)

    @property
    def nx(self) -> int:
        return self.xn.size - 1

    @property
    def ny(self) -> int:
        return self.yn.size - 1

    @property
    def nz(self) -> int:
        return self.zn.size - 1

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class Survey:
    """Observation points (float64 vectors of equal length), z down."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray

    def __post_init__(self):
        self.x = np.ascontiguousarray(self.x, dtype=np.float64)
        self.y = np.ascontiguousarray(self.y, dtype=np.float64)
        self.z = np.ascontiguousarray(self.z, dtype=np.float64)
        assert self.x.shape == self.y.shape == self.z.shape

    @property
    def n(self) -> int:
        return self.x.size

    def take(self, rows) -> "Survey":
        rows = np.asarray(rows)
        return Survey(self.x[rows], self.y[rows], self.z[rows])


@dataclass
class Problem:
    """One workload: geometry, true model and the random draws it needs."""
    name: str
    mesh: Mesh
    obs: Survey
    m: np.ndarray                       # (ncells,) float64 true density contrast
    wdepth: np.ndarray | None = None    # (ncells,) depth weights w (C = w^-2)
    noise_draws: np.ndarray | None = None  # (n,) standard normal draws
    noise_level: float = 0.0            # relative RMS noise (0.01 = 1 %)
    probe_v: np.ndarray | None = None   # (n,) vector for G^T v timings/tests
    cg_tol: float = 0.0
    cg_iters: int = 0
    lambda_factor: float = 1e-2         # lambda = factor * trace(G C G^T) / n
    extra: dict = field(default_factory=dict)


def regular_mesh(nx, ny, nz, dx, dy, dz, x0=0.0, y0=0.0, z0=0.0) -> Mesh:
    return Mesh(x0 + dx * np.arange(nx + 1), y0 + dy * np.arange(ny + 1),
                z0 + dz * np.arange(nz + 1))


def cell_centres(mesh: Mesh):
    """Cell-centre coordinate vectors (xc, yc, zc)."""
    return (0.5 * (mesh.xn[1:] + mesh.xn[:-1]),
            0.5 * (mesh.yn[1:] + mesh.yn[:-1]),
            0.5 * (mesh.zn[1:] + mesh.zn[:-1]))


def _centre_grids(mesh: Mesh):
    xc, yc, zc = cell_centres(mesh)
    return np.meshgrid(xc, yc, zc, indexing="ij")


def depth_weights(mesh: Mesh, z0: float) -> np.ndarray:
    """Li-Oldenburg style depth weight w = (z + z0)^-1 at the cell-centre depth
    below the mesh top, one value per cell (flat C order)."""
    _, _, zc = cell_centres(mesh)
    w_layer = 1.0 / ((zc - mesh.zn[0]) + z0)
    return np.broadcast_to(w_layer, mesh.shape).reshape(-1).copy()


def _uniform_quaternion_rotation(rng) -> np.ndarray:
    """Rotation matrix of a uniformly distributed unit quaternion (Shoemake)."""
    u1, u2, u3 = rng.random(3)
    a = math.sqrt(1.0 - u1)
    b = math.sqrt(u1)
    qx, qy = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    qz, qw = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)],
        [2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)],
        [2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)],
    ])


def ellipsoid_model(mesh: Mesh, rng, count: int, semi_lo: float, semi_hi: float,
                    rho_lo: float = -400.0, rho_hi: float = 400.0) -> np.ndarray:
    """Sum of randomly placed, randomly rotated ellipsoids (cell-centre test);
    overlapping bodies add.  Returns a flat (ncells,) float64 model."""
    X, Y, Z = _centre_grids(mesh)
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    m = np.zeros(P.shape[0])
    lo = np.array([mesh.xn[0], mesh.yn[0], mesh.zn[0]])
    hi = np.array([mesh.xn[-1], mesh.yn[-1], mesh.zn[-1]])
    for _ in range(count):
        c = lo + (hi - lo) * rng.random(3)
        ax = rng.uniform(semi_lo, semi_hi, 3)
        R = _uniform_quaternion_rotation(rng)
        rho = rng.uniform(rho_lo, rho_hi)
        q = (P - c) @ R  # coordinates in the body frame
        inside = np.sum((q / ax) ** 2, axis=1) <= 1.0
        m[inside] += rho
    return m


def dyke_model(mesh: Mesh, vertical: dict, dipping: dict, rho: float) -> np.ndarray:
    """Vertical dyke (axis-aligned box) plus a 45-degree dipping dyke.

    ``vertical``: x0,x1,y0,y1,z0,z1 (half-open box, cell-centre test).
    ``dipping``: xtop (centre-line x at depth ztop), width (horizontal),
    y0,y1, ztop, zbot; the centre line moves +x by one metre per metre of
    depth (45 degrees toward +x)."""
    X, Y, Z = _centre_grids(mesh)
    v = vertical
    vert = ((X >= v["x0"]) & (X < v["x1"]) & (Y >= v["y0"]) & (Y < v["y1"])
            & (Z >= v["z0"]) & (Z < v["z1"]))
    d = dipping
    xc_line = d["xtop"] + (Z - d["ztop"])
    half = 0.5 * d["width"]
    dip = ((X >= xc_line - half) & (X < xc_line + half) & (Y >= d["y0"]) & (Y < d["y1"])
           & (Z >= d["ztop"]) & (Z < d["zbot"]))
    return (rho * (vert | dip)).astype(np.float64).reshape(-1)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def dykes_32x32x16() -> Problem:
    """Tiny plain-FP64 inversion case: 32x32 observation grid on the mesh top
    (50 m spacing, at cell-centre x,y) over a 32x32x16 mesh of 50 m cubes;
    vertical dyke 100x400x500 m plus a 45-degree dipping dyke, +300 kg/m^3;
    1 % Gaussian noise (seed 1); w = (z + 25 m)^-1; CG to 1e-6."""
    mesh = regular_mesh(32, 32, 16, 50.0, 50.0, 50.0)
    m = dyke_model(
        mesh,
        vertical=dict(x0=500.0, x1=600.0, y0=600.0, y1=1000.0, z0=50.0, z1=550.0),
        dipping=dict(xtop=1000.0, width=100.0, y0=600.0, y1=1000.0, ztop=50.0, zbot=550.0),
        rho=300.0)
    xc, yc, _ = cell_centres(mesh)
    OX, OY = np.meshgrid(xc, yc, indexing="ij")
    obs = Survey(OX.ravel(), OY.ravel(), np.zeros(OX.size))
    rng = np.random.default_rng(1)
    return Problem("dykes_32x32x16", mesh, obs, m, wdepth=depth_weights(mesh, 25.0),
                   noise_draws=rng.standard_normal(obs.n), noise_level=0.01,
                   cg_tol=1e-6, cg_iters=0)


def ellipsoids_100x100x50() -> Problem:
    """Forward/adjoint case: 100x100 observation grid (25 m spacing, cell-centre
    x,y) at random heights U[0,50] m over a 100x100x50 mesh of 25 m cubes;
    density = 20 random ellipsoids, contrast U[-400,400] kg/m^3 (seed 0);
    probe vector v ~ N(0,1) (seed 2)."""
    mesh = regular_mesh(100, 100, 50, 25.0, 25.0, 25.0)
    rng = np.random.default_rng(0)
    xc, yc, _ = cell_centres(mesh)
    OX, OY = np.meshgrid(xc, yc, indexing="ij")
    h = rng.uniform(0.0, 50.0, OX.size)
    obs = Survey(OX.ravel(), OY.ravel(), mesh.zn[0] - h)
    m = ellipsoid_model(mesh, rng, 20, 50.0, 625.0)
    v = np.random.default_rng(2).standard_normal(obs.n)
    return Problem("ellipsoids_100x100x50", mesh, obs, m, probe_v=v)


def smoothed_box_models(mesh: Mesh, count: int = 64, first_seed: int = 100) -> np.ndarray:
    """Block of density models for the multi-model forward: model j (seed
    first_seed + j) = 5 random axis-aligned boxes (sides U[75,750] m, contrast
    U[-400,400]) plus N(0,1) white noise smoothed by a 3-D Gaussian of sigma =
    3 cells (zero boundary), scaled to standard deviation 50 kg/m^3.
    Returns (ncells, count) float64, model index fastest."""
    from scipy.ndimage import gaussian_filter
    X, Y, Z = _centre_grids(mesh)
    lo = np.array([mesh.xn[0], mesh.yn[0], mesh.zn[0]])
    hi = np.array([mesh.xn[-1], mesh.yn[-1], mesh.zn[-1]])
    out = np.empty((mesh.ncells, count))
    for j in range(count):
        rng = np.random.default_rng(first_seed + j)
        mj = np.zeros(mesh.shape)
        for _ in range(5):
            c = lo + (hi - lo) * rng.random(3)
            side = rng.uniform(75.0, 750.0, 3)
            rho = rng.uniform(-400.0, 400.0)
            inside = ((np.abs(X - c[0]) < side[0] / 2) & (np.abs(Y - c[1]) < side[1] / 2)
                      & (np.abs(Z - c[2]) < side[2] / 2))
            mj[inside] += rho
        noise = gaussian_filter(rng.standard_normal(mesh.shape), sigma=3.0,
                                mode="constant", cval=0.0)
        noise *= 50.0 / noise.std()
        out[:, j] = (mj + noise).reshape(-1)
    return out


def paper_scale(n_obs: int = 178_797) -> Problem:
    """Paper-scale case: 178,797 observations scattered uniformly over a
    15x15 km area (seed 4) at heights of a synthetic Gaussian-bump topography
    (max 300 m) over a 150x150x147 mesh of 100x100x70 m cells (3,307,500
    prisms); two +300 kg/m^3 dykes plus 10 random ellipsoids; 2 % noise;
    data-space CG with 50 iterations."""
    mesh = regular_mesh(150, 150, 147, 100.0, 100.0, 70.0)
    rng = np.random.default_rng(4)
    ox = rng.uniform(0.0, 15000.0, n_obs)
    oy = rng.uniform(0.0, 15000.0, n_obs)
    h = np.zeros(n_obs)
    for _ in range(6):
        amp = rng.uniform(100.0, 300.0)
        sig = rng.uniform(1000.0, 3000.0)
        cx, cy = rng.uniform(0.0, 15000.0, 2)
        h += amp * np.exp(-((ox - cx) ** 2 + (oy - cy) ** 2) / (2 * sig * sig))
    h *= 300.0 / h.max()
    obs = Survey(ox, oy, mesh.zn[0] - h)
    m = dyke_model(
        mesh,
        vertical=dict(x0=4000.0, x1=4300.0, y0=5500.0, y1=9500.0, z0=500.0, z1=3500.0),
        dipping=dict(xtop=9000.0, width=300.0, y0=5500.0, y1=9500.0, ztop=500.0, zbot=3500.0),
        rho=300.0)
    m += ellipsoid_model(mesh, rng, 10, 300.0, 2500.0)
    noise = rng.standard_normal(n_obs)
    v = np.random.default_rng(40).standard_normal(n_obs)
    return Problem("paper_scale", mesh, obs, m, wdepth=depth_weights(mesh, 25.0),
                   noise_draws=noise, noise_level=0.02, probe_v=v, cg_iters=50)


def serving_stream(n_requests: int = 200, mean_gap_s: float = 0.5, seed: int = 5,
                   n_lo: int = 1000, n_hi: int = 40000,
                   cells_lo: int = 50_000, cells_hi: int = 800_000):
    """Serving stream: Poisson arrivals (exponential gaps, mean 0.5 s), each a
    forward or an inversion request (p = 0.5) with a log-uniform observation
    count in [1k, 40k] (regular sqrt(N) x sqrt(N) grid, 25 m spacing, on the
    mesh top) and a log-uniform cell count in [50k, 800k] (nx = ny = 2 nz, 25 m
    cubes) holding a random vertical and a random dipping dyke (+300 kg/m^3);
    1 % noise; inversions run CG to 1e-6 (at most 200 iterations).

    Returns a list of dicts: arrival time, kind, and a zero-argument callable
    ``build()`` that materialises the request's Problem."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for r in range(n_requests):
        t += rng.exponential(mean_gap_s)
        kind = "inversion" if rng.random() < 0.5 else "forward"
        n = math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))
        cells = math.exp(rng.uniform(math.log(cells_lo), math.log(cells_hi)))
        sub_seed = int(rng.integers(0, 2**31 - 1))
        reqs.append(dict(t=t, kind=kind, n_target=n, cells_target=cells, seed=sub_seed,
                         build=_stream_request_builder(kind, n, cells, sub_seed)))
    return reqs


def _stream_request_builder(kind, n_target, cells_target, seed):
    def build() -> Problem:
        rng = np.random.default_rng(seed)
        nz = max(2, int(round((cells_target / 4.0) ** (1.0 / 3.0))))
        nx = ny = 2 * nz
        mesh = regular_mesh(nx, ny, nz, 25.0, 25.0, 25.0)
        g = max(2, int(round(math.sqrt(n_target))))
        ext = nx * 25.0
        off = 0.5 * (ext - g * 25.0)
        c = off + 12.5 + 25.0 * np.arange(g)
        OX, OY = np.meshgrid(c, c, indexing="ij")
        obs = Survey(OX.ravel(), OY.ravel(), np.zeros(OX.size))
        depth = nz * 25.0
        vx = rng.uniform(0.15, 0.45) * ext
        vw = rng.uniform(50.0, 150.0)
        y0 = rng.uniform(0.1, 0.4) * ext
        y1 = y0 + rng.uniform(0.3, 0.5) * ext
        z0 = rng.uniform(0.05, 0.2) * depth
        z1 = z0 + rng.uniform(0.3, 0.6) * depth
        m = dyke_model(
            mesh,
            vertical=dict(x0=vx, x1=vx + vw, y0=y0, y1=y1, z0=z0, z1=z1),
            dipping=dict(xtop=rng.uniform(0.55, 0.75) * ext, width=rng.uniform(50.0, 150.0),
                         y0=y0, y1=y1, ztop=z0, zbot=z1),
            rho=300.0)
        return Problem(f"stream-{kind}", mesh, obs, m, wdepth=depth_weights(mesh, 25.0),
                       noise_draws=rng.standard_normal(obs.n), noise_level=0.01,
                       cg_tol=1e-6 if kind == "inversion" else 0.0,
                       cg_iters=200 if kind == "inversion" else 0,
                       extra=dict(kind=kind))
    return build


def regional_sections(seed: int = 45, nx: int = 10, ny: int = 18, nz: int = 6,
                      n_obs: int = 320, cell: float = 100.0, nsec: int = 3) -> Problem:
    """Small regional survey for the section workflow, shaped like the paper's
    regional example (a domain longer north-south (y) than east-west, about
    1.7 : 1, divided into adjoining sections along y): a regular mesh of
    ``cell``-metre cubes, ``n_obs`` stations on a jittered grid over the
    footprint at heights U[0, 30] m, three random ellipsoids (contrast
    U[-400, 400] kg/m^3, semi-axes 0.1-0.45 of the width, so bodies straddle
    section boundaries), and a regional field: a second-degree polynomial in
    the normalised station coordinates u = (x - xc) / (width / 2),
    w = (y - yc) / (length / 2) with coefficients U[-1, 1] x 3e-5 m/s^2 (about
    3 mGal, larger than the local anomaly).  ``extra``: ysplit (nsec equal
    sections of whole cell rows) and regional_coef (constant, u, w, u^2, u w,
    w^2).  1 % noise draws; w = (z + 25 m)^-1."""
    rng = np.random.default_rng(seed)
    mesh = regular_mesh(nx, ny, nz, cell, cell, cell)
    wx, wy = nx * cell, ny * cell
    gx = max(2, int(round(math.sqrt(n_obs * wx / wy))))
    gy = max(2, -(-n_obs // gx))
    ox = (np.arange(gx * gy) % gx + 0.5) * (wx / gx)
    oy = (np.arange(gx * gy) // gx + 0.5) * (wy / gy)
    keep = rng.permutation(gx * gy)[:n_obs]
    ox = ox[keep] + rng.uniform(-0.3, 0.3, n_obs) * (wx / gx)
    oy = oy[keep] + rng.uniform(-0.3, 0.3, n_obs) * (wy / gy)
    oz = mesh.zn[0] - rng.uniform(0.0, 30.0, n_obs)
    obs = Survey(ox, oy, oz)
    m = ellipsoid_model(mesh, rng, 3, 0.1 * wx, 0.45 * wx)
    coef = rng.uniform(-1.0, 1.0, 6) * 3e-5
    ysplit = np.round(np.linspace(0, ny, nsec + 1)).astype(int)
    return Problem(f"regional_sections-{seed}", mesh, obs, m, wdepth=depth_weights(mesh, 25.0),
                   noise_draws=rng.standard_normal(n_obs), noise_level=0.01,
                   extra=dict(ysplit=ysplit, regional_coef=coef,
                              centre=(0.5 * wx, 0.5 * wy), half=(0.5 * wx, 0.5 * wy)))


def regional_field(p: Problem) -> np.ndarray:
    """The regional polynomial of ``regional_sections`` at the stations."""
    c = p.extra["regional_coef"]
    u = (p.obs.x - p.extra["centre"][0]) / p.extra["half"][0]
    w = (p.obs.y - p.extra["centre"][1]) / p.extra["half"][1]
    return c[0] + c[1] * u + c[2] * w + c[3] * u * u + c[4] * u * w + c[5] * w * w


def random_case(seed: int, nx: int, ny: int, nz: int, n_obs: int, *,
                spacing=(10.0, 60.0), rectilinear: bool = True, height_max: float = 50.0,
                on_nodes: int = 0, on_top: int = 0, model: str = "noise") -> Problem:
    """Random small case for parity tests: rectilinear node spacings in
    ``spacing`` (or uniform), observations scattered over the mesh footprint
    widened by 20 %, heights U[0, height_max].  ``on_nodes`` observations are
    snapped to node (x, y) positions and ``on_top`` to the mesh top (z = zn[0]),
    exercising the singular limits.  ``model``: "noise" (N(0, 100^2)) or
    "blocky" (ellipsoids)."""
    rng = np.random.default_rng(seed)

    def nodes(n):
        if rectilinear:
            return np.concatenate([[0.0], np.cumsum(rng.uniform(*spacing, n))])
        return np.arange(n + 1) * 0.5 * (spacing[0] + spacing[1])

    mesh = Mesh(nodes(nx) - 20.0, nodes(ny) + 5.0, nodes(nz))
    wx = mesh.xn[-1] - mesh.xn[0]
    wy = mesh.yn[-1] - mesh.yn[0]
    ox = rng.uniform(mesh.xn[0] - 0.1 * wx, mesh.xn[-1] + 0.1 * wx, n_obs)
    oy = rng.uniform(mesh.yn[0] - 0.1 * wy, mesh.yn[-1] + 0.1 * wy, n_obs)
    oz = mesh.zn[0] - rng.uniform(0.0, height_max, n_obs)
    k = min(on_nodes, n_obs)
    if k:
        ox[:k] = mesh.xn[rng.integers(0, nx + 1, k)]
        oy[:k] = mesh.yn[rng.integers(0, ny + 1, k)]
    k2 = min(on_top, n_obs)
    if k2:
        oz[:k2] = mesh.zn[0]
    obs = Survey(ox, oy, oz)
    if model == "noise":
        m = 100.0 * rng.standard_normal(mesh.ncells)
    else:
        m = ellipsoid_model(mesh, rng, 4, 0.1 * wx, 0.5 * wx)
    wdepth = depth_weights(mesh, 25.0)
    return Problem(f"random-{seed}", mesh, obs, m, wdepth=wdepth,
                   probe_v=rng.standard_normal(n_obs),
                   noise_draws=rng.standard_normal(n_obs), noise_level=0.01)
