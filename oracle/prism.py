"""FP64 CPU oracle: the prism vertical-attraction kernel and the forward /
adjoint operators built from it.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only the tests, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the GPU library.

Everything is plain float64 NumPy, written to be checked against the paper by
eye:

* ``psi`` is the corner function of Eq. 2 with R from Eq. 3.
* ``sensitivity_literal`` / ``forward_literal`` evaluate Eq. 1 prism by prism
  (8 corners, vertex parity sigma = (-1)^(p+q+r)) and superpose with Eq. 4-6.
* ``forward`` / ``adjoint`` / ``sensitivity_row`` regroup the same sum by mesh
  node: every corner of every prism is a node of the mesh, so
  ``d_o = gamma * sum_nodes Psi(node - o) * W_node`` with the node weight
  ``W = B m`` collecting the parities of the (up to 8) cells meeting at the
  node.  This is an exact regrouping of Eq. 1 and 5 (checked against the
  literal form in the tests), used because the literal form is 8x slower.

Readings of the paper adopted here (each also listed in the design notes):

* Coordinates in Psi are corner minus observation, z positive down, vertex
  index 1 = the smaller coordinate.  With sigma as printed this gives gz > 0
  (downward pull) for positive density below the observation; the Bouguer-slab
  test pins it.
* Singular limits (the paper only says "singularity-robust"): the x-log term is
  0 when x = 0, the y-log term is 0 when y = 0, the atan term is 0 when z = 0.
  Each is the continuous limit of the expression.
* ln(R + y) for y < 0 is evaluated as ln((x^2 + z^2) / (R - y)), the same
  number written without the cancellation of R + y (R^2 - y^2 = x^2 + z^2);
  likewise ln(R + x) for x < 0.
"""
from __future__ import annotations

import numpy as np

GAMMA = 6.674e-11  # gravitational constant used by the paper's workloads, SI


def psi(x, y, z):
    """Corner function Psi(x, y, z) of Eq. 2, R = sqrt(x^2 + y^2 + z^2) (Eq. 3).

    Arguments are corner-minus-observation coordinates (broadcastable float64
    arrays).  Returns z*atan(xy/(zR)) - x*ln(R+y) - y*ln(R+x) with the limit
    conventions described in the module docstring."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    R = np.sqrt(x * x + y * y + z * z)
    with np.errstate(divide="ignore", invalid="ignore"):
        t_atan = np.where(z != 0.0, z * np.arctan((x * y) / (z * R)), 0.0)
        r_plus_y = np.where(y >= 0.0, R + y, (x * x + z * z) / (R - y))
        r_plus_x = np.where(x >= 0.0, R + x, (y * y + z * z) / (R - x))
        t_x = np.where(x != 0.0, x * np.log(r_plus_y), 0.0)
        t_y = np.where(y != 0.0, y * np.log(r_plus_x), 0.0)
    return t_atan - t_x - t_y


# --------------------------------------------------------------------------
# Literal per-prism form (Eq. 1, 4-6): small inputs only
# --------------------------------------------------------------------------

def prism_corner_sum(x1, x2, y1, y2, z1, z2):
    """sum_{p,q,r in {1,2}} (-1)^(p+q+r) Psi(x_p, y_q, z_r) for one prism whose
    corners relative to the observation are (x1|x2, y1|y2, z1|z2) (Eq. 1
    without the factor gamma*rho).  Broadcasts over array arguments."""
    xs, ys, zs = (x1, x2), (y1, y2), (z1, z2)
    total = 0.0
    for p in (1, 2):
        for q in (1, 2):
            for r in (1, 2):
                sigma = (-1.0) ** (p + q + r)
                total = total + sigma * psi(xs[p - 1], ys[q - 1], zs[r - 1])
    return total


def sensitivity_literal(mesh, obs) -> np.ndarray:
    """Dense sensitivity matrix G (n x M), G[o, k] = gamma * corner sum of
    prism k seen from observation o (Eq. 1, 5, 6).  Flat cell index
    k = (i*ny + j)*nz + kz."""
    nx, ny, nz = mesh.nx, mesh.ny, mesh.nz
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    G = np.empty((obs.n, mesh.ncells))
    for o in range(obs.n):
        G[o] = GAMMA * prism_corner_sum(
            mesh.xn[I] - obs.x[o], mesh.xn[I + 1] - obs.x[o],
            mesh.yn[J] - obs.y[o], mesh.yn[J + 1] - obs.y[o],
            mesh.zn[K] - obs.z[o], mesh.zn[K + 1] - obs.z[o])
    return G


def forward_literal(mesh, obs, m) -> np.ndarray:
    """d = G m with G from ``sensitivity_literal`` (Eq. 6)."""
    return sensitivity_literal(mesh, obs) @ np.asarray(m, dtype=np.float64)


# --------------------------------------------------------------------------
# Node-shared regrouping of the same sum
# --------------------------------------------------------------------------

def node_weights(mesh, m) -> np.ndarray:
    """W = B m on the (nx+1, ny+1, nz+1) node grid.

    Node (a, b, c) is corner (p, q, r) of cell (a-p+1, b-q+1, c-r+1) for
    p, q, r in {1, 2}; it collects sigma_pqr * m of every such cell that
    exists (Eq. 1 summed over cells as in Eq. 5)."""
    mm = np.asarray(m, dtype=np.float64).reshape(mesh.shape)
    W = np.zeros((mesh.nx + 1, mesh.ny + 1, mesh.nz + 1))
    for p in (1, 2):
        for q in (1, 2):
            for r in (1, 2):
                sigma = (-1.0) ** (p + q + r)
                # cell i has its p-corner at node a = i + p - 1
                W[p - 1:p - 1 + mesh.nx, q - 1:q - 1 + mesh.ny, r - 1:r - 1 + mesh.nz] += sigma * mm
    return W


def node_weights_transpose(mesh, P) -> np.ndarray:
    """B^T P: per cell, sum_{pqr} sigma_pqr * P(corner node) (flat, C order)."""
    P = np.asarray(P, dtype=np.float64).reshape(mesh.nx + 1, mesh.ny + 1, mesh.nz + 1)
    out = np.zeros(mesh.shape)
    for p in (1, 2):
        for q in (1, 2):
            for r in (1, 2):
                sigma = (-1.0) ** (p + q + r)
                out += sigma * P[p - 1:p - 1 + mesh.nx, q - 1:q - 1 + mesh.ny, r - 1:r - 1 + mesh.nz]
    return out.reshape(-1)


def psi_nodes(mesh, xo: float, yo: float, zo: float) -> np.ndarray:
    """Psi(node - observation) at every mesh node, shape (nx+1, ny+1, nz+1)."""
    x = (mesh.xn - xo)[:, None, None]
    y = (mesh.yn - yo)[None, :, None]
    z = (mesh.zn - zo)[None, None, :]
    return psi(x, y, z)


def sensitivity_row(mesh, xo: float, yo: float, zo: float) -> np.ndarray:
    """Row o of G (length M): gamma * B^T Psi_nodes(o)."""
    return GAMMA * node_weights_transpose(mesh, psi_nodes(mesh, xo, yo, zo))


def forward(mesh, obs, m, rows=None) -> np.ndarray:
    """d = G m (Eq. 6) for all observations, or for the listed ``rows``."""
    W = node_weights(mesh, m)
    rows = np.arange(obs.n) if rows is None else np.asarray(rows)
    d = np.empty(rows.size)
    for t, o in enumerate(rows):
        d[t] = GAMMA * np.sum(psi_nodes(mesh, obs.x[o], obs.y[o], obs.z[o]) * W)
    return d


def forward_multi(mesh, obs, models, rows=None) -> np.ndarray:
    """D = G M for a block of models (M x K, model index fastest): Psi is
    evaluated once per (observation, node) and contracted with every model's
    node weights.  Returns (n_rows, K)."""
    models = np.asarray(models, dtype=np.float64)
    K = models.shape[1]
    Wk = np.stack([node_weights(mesh, models[:, j]).reshape(-1) for j in range(K)], axis=1)
    rows = np.arange(obs.n) if rows is None else np.asarray(rows)
    D = np.empty((rows.size, K))
    for t, o in enumerate(rows):
        D[t] = GAMMA * (psi_nodes(mesh, obs.x[o], obs.y[o], obs.z[o]).reshape(-1) @ Wk)
    return D


def adjoint(mesh, obs, v) -> np.ndarray:
    """g = G^T v: gamma * B^T (sum_o v_o Psi_nodes(o))."""
    v = np.asarray(v, dtype=np.float64)
    P = np.zeros((mesh.nx + 1, mesh.ny + 1, mesh.nz + 1))
    for o in range(obs.n):
        P += v[o] * psi_nodes(mesh, obs.x[o], obs.y[o], obs.z[o])
    return GAMMA * node_weights_transpose(mesh, P)


def adjoint_cells(mesh, obs, v, cells) -> np.ndarray:
    """Selected entries (G^T v)_k, each computed from its own 8 corners for all
    observations (used to check large adjoints entry by entry)."""
    v = np.asarray(v, dtype=np.float64)
    cells = np.asarray(cells)
    i, rem = np.divmod(cells, mesh.ny * mesh.nz)
    j, k = np.divmod(rem, mesh.nz)
    out = np.empty(cells.size)
    for t in range(cells.size):
        col = GAMMA * prism_corner_sum(
            mesh.xn[i[t]] - obs.x, mesh.xn[i[t] + 1] - obs.x,
            mesh.yn[j[t]] - obs.y, mesh.yn[j[t] + 1] - obs.y,
            mesh.zn[k[t]] - obs.z, mesh.zn[k[t] + 1] - obs.z)
        out[t] = np.dot(col, v)
    return out


def weighted_row_sumsq(mesh, obs, cov, rows=None) -> np.ndarray:
    """Per observation o: sum_k C_k G_ok^2, i.e. the diagonal of G C G^T.
    Its sum over all observations is trace(G C G^T)."""
    cov = np.asarray(cov, dtype=np.float64)
    rows = np.arange(obs.n) if rows is None else np.asarray(rows)
    out = np.empty(rows.size)
    for t, o in enumerate(rows):
        g = sensitivity_row(mesh, obs.x[o], obs.y[o], obs.z[o])
        out[t] = np.dot(cov * g, g)
    return out


# --------------------------------------------------------------------------
# Rounding-error scales (magnitudes of the summed terms), used by the tests to
# derive tolerances for low-precision evaluations of the same sums.
# --------------------------------------------------------------------------

def edge_terms(mesh, xo: float, yo: float, zo: float) -> np.ndarray:
    """S(a, b, k) = Psi(node (a, b, k+1) - o) - Psi(node (a, b, k) - o): the
    sum of Eq. 1's vertex terms over the two ends of each vertical mesh edge
    segment, shape (nx+1, ny+1, nz)."""
    P = psi_nodes(mesh, xo, yo, zo)
    return P[:, :, 1:] - P[:, :, :-1]


def forward_abs_scale(mesh, obs, m, rows) -> np.ndarray:
    """gamma * sum over vertical edge segments of |S| * |sum of the up to four
    adjacent cells' parity-weighted densities| per observation row: the size of
    the terms a segment-wise evaluation of G m adds up."""
    mm = np.asarray(m, dtype=np.float64).reshape(mesh.shape)
    W2 = np.zeros((mesh.nx + 1, mesh.ny + 1, mesh.nz))
    for p in (0, 1):
        for q in (0, 1):
            W2[p:p + mesh.nx, q:q + mesh.ny, :] += (-1.0) ** (p + q) * mm
    out = np.empty(len(rows))
    for t, o in enumerate(rows):
        out[t] = GAMMA * np.sum(np.abs(edge_terms(mesh, obs.x[o], obs.y[o], obs.z[o]) * W2))
    return out


def adjoint_abs_scale(mesh, obs, v, cells) -> np.ndarray:
    """gamma * sum_o |v_o| * sum over the cell's four vertical edges of |S|:
    the size of the terms an edge-wise evaluation of (G^T v)_cell adds up."""
    v = np.asarray(v, dtype=np.float64)
    cells = np.asarray(cells)
    i, rem = np.divmod(cells, mesh.ny * mesh.nz)
    j, k = np.divmod(rem, mesh.nz)
    out = np.empty(cells.size)
    for t in range(cells.size):
        acc = np.zeros(obs.n)
        for p in (0, 1):
            for q in (0, 1):
                x = mesh.xn[i[t] + p] - obs.x
                y = mesh.yn[j[t] + q] - obs.y
                acc += np.abs(psi(x, y, mesh.zn[k[t] + 1] - obs.z) - psi(x, y, mesh.zn[k[t]] - obs.z))
        out[t] = GAMMA * np.dot(np.abs(v), acc)
    return out


def adjoint_abs_scale_corners(mesh, obs, v, cells) -> np.ndarray:
    """gamma * sum_o |v_o| * sum over the cell's 8 corners of |Psi|: the size
    of the terms a corner-wise (node) evaluation of (G^T v)_cell adds up."""
    v = np.asarray(v, dtype=np.float64)
    cells = np.asarray(cells)
    i, rem = np.divmod(cells, mesh.ny * mesh.nz)
    j, k = np.divmod(rem, mesh.nz)
    out = np.empty(cells.size)
    for t in range(cells.size):
        acc = np.zeros(obs.n)
        for p in (0, 1):
            for q in (0, 1):
                for r in (0, 1):
                    acc += np.abs(psi(mesh.xn[i[t] + p] - obs.x, mesh.yn[j[t] + q] - obs.y,
                                      mesh.zn[k[t] + r] - obs.z))
        out[t] = GAMMA * np.dot(np.abs(v), acc)
    return out
