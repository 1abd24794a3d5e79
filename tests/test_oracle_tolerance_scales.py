"""Pins of the oracle's rounding-scale helpers (``prism.edge_terms``,
``forward_abs_scale``, ``adjoint_abs_scale``, ``adjoint_abs_scale_corners``).
CPU only.

These helpers do not compute reference values: they give the summed
magnitude of the terms a low-precision evaluation adds up, from which the GPU
tests derive condition-aware tolerances.  A wrong index, a missing |v|, a
wrong density-parity stencil or a stray factor would silently loosen or
tighten those tests, so each helper is pinned two ways:

* against a hand-indexed evaluation on one- and two-cell meshes, with Psi of
  Eq. 2 evaluated to 40 digits by mpmath (independent of the oracle's NumPy
  ``psi``), written out edge by edge / corner by corner;
* by inequalities any correct magnitude sum obeys on random cases: it bounds
  the absolute value of the sum it describes (triangle inequality), and the
  edge scale never exceeds the corner scale (each edge term is the difference
  of two corner terms).
"""
import mpmath as mp
import numpy as np

from oracle import GAMMA, prism
from workloads import Mesh, Survey, random_case

mp.mp.dps = 40


def _psi_mp(x, y, z):
    """Eq. 2 with the limits of the oracle (x = 0, y = 0, z = 0 terms vanish),
    40 digits."""
    x, y, z = mp.mpf(x), mp.mpf(y), mp.mpf(z)
    R = mp.sqrt(x * x + y * y + z * z)
    t = z * mp.atan(x * y / (z * R)) if z != 0 else mp.mpf(0)
    tx = x * mp.log(R + y) if x != 0 else mp.mpf(0)
    ty = y * mp.log(R + x) if y != 0 else mp.mpf(0)
    return t - tx - ty


def _edge_mp(X, Y, z1, z2, o):
    """S = Psi(X - xo, Y - yo, z2 - zo) - Psi(X - xo, Y - yo, z1 - zo)."""
    xo, yo, zo = o
    return _psi_mp(X - xo, Y - yo, z2 - zo) - _psi_mp(X - xo, Y - yo, z1 - zo)


def _two_cell_mesh():
    # cells (0, 0, 0) and (1, 0, 0): unequal widths so that a swapped index shows
    return Mesh(np.array([-30.0, 45.0, 70.0]), np.array([10.0, 95.0]), np.array([5.0, 65.0]))


def _stations():
    # above the first cell, above the second, outside the footprint, on the top face
    return Survey(np.array([0.0, 60.0, 300.0, 44.0]), np.array([50.0, 20.0, -140.0, 96.0]),
                  np.array([-12.0, -3.0, -40.0, 5.0]))


def test_edge_terms_parity_sum_is_the_prism_corner_sum():
    """sum_{p,q} (-1)^(p+q) S(i+p, j+q, k) is Eq. 1's 8-corner sum of cell
    (i, j, k): catches a wrong edge index, a reversed z difference or a wrong
    node offset in edge_terms."""
    p = random_case(31, 5, 4, 6, 7, on_nodes=2, on_top=2)
    mesh, obs = p.mesh, p.obs
    for o in range(obs.n):
        S = prism.edge_terms(mesh, obs.x[o], obs.y[o], obs.z[o])
        assert S.shape == (mesh.nx + 1, mesh.ny + 1, mesh.nz)
        par = S[:-1, :-1, :] - S[1:, :-1, :] - S[:-1, 1:, :] + S[1:, 1:, :]
        for i in range(mesh.nx):
            for j in range(mesh.ny):
                for k in range(mesh.nz):
                    lit = prism.prism_corner_sum(
                        mesh.xn[i] - obs.x[o], mesh.xn[i + 1] - obs.x[o],
                        mesh.yn[j] - obs.y[o], mesh.yn[j + 1] - obs.y[o],
                        mesh.zn[k] - obs.z[o], mesh.zn[k + 1] - obs.z[o])
                    mag = np.abs(S[i:i + 2, j:j + 2, k]).sum()
                    assert abs(par[i, j, k] - lit) <= 1e-12 * mag


def test_edge_terms_against_mpmath():
    mesh, obs = _two_cell_mesh(), _stations()
    for o in range(obs.n):
        S = prism.edge_terms(mesh, obs.x[o], obs.y[o], obs.z[o])
        for a in range(3):
            for b in range(2):
                ref = _edge_mp(mesh.xn[a], mesh.yn[b], mesh.zn[0], mesh.zn[1],
                               (obs.x[o], obs.y[o], obs.z[o]))
                assert abs(S[a, b, 0] - float(ref)) <= 1e-12 * (abs(float(ref)) + 1.0)


def test_forward_abs_scale_2x2_cells_by_hand():
    """Four cells (i, j) in one layer with densities m_ij: the (x, y) parity
    stencil gives the node-column weights written out below (node column
    (a, b) sees the cells with corners there), and the scale is
    gamma * sum over the 9 columns of |W2| * |S|."""
    mesh = Mesh(np.array([-30.0, 45.0, 70.0]), np.array([10.0, 95.0, 130.0]),
                np.array([5.0, 65.0]))
    obs = _stations()
    m00, m01, m10, m11 = 250.0, -110.0, 40.0, 310.0
    W2 = {(0, 0): m00, (0, 1): m01 - m00, (0, 2): -m01,
          (1, 0): m10 - m00, (1, 1): m11 - m10 - m01 + m00, (1, 2): m01 - m11,
          (2, 0): -m10, (2, 1): m10 - m11, (2, 2): m11}
    m = np.array([m00, m01, m10, m11])          # flat (i*ny + j)*nz + k order
    got = prism.forward_abs_scale(mesh, obs, m, np.arange(obs.n))
    for o in range(obs.n):
        oo = (obs.x[o], obs.y[o], obs.z[o])
        ref = sum(abs(w) * abs(_edge_mp(mesh.xn[a], mesh.yn[b], mesh.zn[0], mesh.zn[1], oo))
                  for (a, b), w in W2.items())
        assert abs(got[o] - GAMMA * float(ref)) <= 1e-12 * GAMMA * float(ref)


def test_adjoint_abs_scales_by_hand():
    """Per cell: gamma * sum_o |v_o| sum over the cell's 4 vertical edges of |S|
    (edge scale) and of its 8 corners of |Psi| (corner scale); v of mixed sign
    (a missing |.| shows), two cells (a wrong cell index shows)."""
    mesh, obs = _two_cell_mesh(), _stations()
    v = np.array([1.5, -0.25, 2.0, -3.0])
    e = prism.adjoint_abs_scale(mesh, obs, v, np.array([0, 1]))
    c = prism.adjoint_abs_scale_corners(mesh, obs, v, np.array([0, 1]))
    for cell in (0, 1):
        ref_e = mp.mpf(0)
        ref_c = mp.mpf(0)
        for o in range(obs.n):
            oo = (obs.x[o], obs.y[o], obs.z[o])
            for a in (cell, cell + 1):
                for b in (0, 1):
                    ref_e += abs(v[o]) * abs(_edge_mp(mesh.xn[a], mesh.yn[b], mesh.zn[0],
                                                       mesh.zn[1], oo))
                    for kz in (0, 1):
                        ref_c += abs(v[o]) * abs(_psi_mp(mesh.xn[a] - oo[0], mesh.yn[b] - oo[1],
                                                         mesh.zn[kz] - oo[2]))
        assert abs(e[cell] - GAMMA * float(ref_e)) <= 1e-12 * GAMMA * float(ref_e)
        assert abs(c[cell] - GAMMA * float(ref_c)) <= 1e-12 * GAMMA * float(ref_c)


def test_adjoint_abs_scale_cell_index_order():
    """A cell deep inside a 3 x 4 x 5 mesh: the scale is that of its own
    edges, i.e. the same number as on a one-cell mesh cut out around it
    (catches a transposed (i, j, k) decomposition of the flat index)."""
    p = random_case(32, 3, 4, 5, 6)
    v = p.probe_v
    i, j, k = 1, 2, 3
    cell = (i * p.mesh.ny + j) * p.mesh.nz + k
    one = Mesh(p.mesh.xn[i:i + 2], p.mesh.yn[j:j + 2], p.mesh.zn[k:k + 2])
    for fn in (prism.adjoint_abs_scale, prism.adjoint_abs_scale_corners):
        got = fn(p.mesh, p.obs, v, np.array([cell]))[0]
        ref = fn(one, p.obs, v, np.array([0]))[0]
        assert got == ref


def test_scales_bound_the_sums_they_describe():
    """Triangle inequality on random cases (noise density, random-sign v):
    |G m|_o <= forward scale, |G^T v|_cell <= edge scale <= corner scale."""
    for seed, shape in ((33, (6, 5, 4)), (34, (3, 7, 9))):
        p = random_case(seed, *shape, 40, on_nodes=4, on_top=4)
        rows = np.arange(p.obs.n)
        d = prism.forward(p.mesh, p.obs, p.m)
        fs = prism.forward_abs_scale(p.mesh, p.obs, p.m, rows)
        assert np.all(np.abs(d) <= fs * (1 + 1e-12))
        cells = np.arange(p.mesh.ncells)
        g = prism.adjoint_cells(p.mesh, p.obs, p.probe_v, cells)
        es = prism.adjoint_abs_scale(p.mesh, p.obs, p.probe_v, cells)
        cs = prism.adjoint_abs_scale_corners(p.mesh, p.obs, p.probe_v, cells)
        assert np.all(np.abs(g) <= es * (1 + 1e-12))
        assert np.all(es <= cs * (1 + 1e-12))
        # and none of them is wildly loose for a sign-definite v and density
        # of one sign: then every observation's contribution adds up
        vpos = np.abs(p.probe_v)
        gpos = prism.adjoint_cells(p.mesh, p.obs, vpos, cells)
        assert np.all(gpos > 0)
