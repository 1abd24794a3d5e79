"""FP64 CPU oracle for the data-space inversion (paper Section 2.2, Eq. 7-11).

TEST INFRASTRUCTURE ONLY (see ``oracle.prism``).  Plain NumPy / SciPy float64.

Notation follows the paper: W_d = lambda * I (uniform data covariance
delta, read as lambda), W_m = C = diag(w^-2) built from the depth weights w
(the penalty (m - m_ref)^T W_m^-1 (m - m_ref) of Eq. 7 with W_m^-1 =
diag(w^2)), delta_d = d_obs - G m_ref, and the data-space solution of Eq. 11

    delta_m = C G^T (G C G^T + lambda I)^-1 delta_d .
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from . import prism


def covariance_from_weights(wdepth) -> np.ndarray:
    """C = W_m = diag(w^-2) as a vector (the depth-weighting reading of Eq. 7)."""
    w = np.asarray(wdepth, dtype=np.float64)
    return 1.0 / (w * w)


def lambda_rule(trace: float, n: int, factor: float = 1e-2) -> float:
    """lambda = factor * trace(G C G^T) / n (the workloads' choice of delta)."""
    return factor * trace / n


def add_noise(d_clean, draws, level) -> np.ndarray:
    """d_obs = d_clean + level * RMS(d_clean) * draws (relative Gaussian noise
    as in the paper's synthetic tests, Section 4.1)."""
    d_clean = np.asarray(d_clean, dtype=np.float64)
    rms = np.sqrt(np.mean(d_clean * d_clean))
    return d_clean + level * rms * np.asarray(draws, dtype=np.float64)


# --------------------------------------------------------------------------
# Dense forms (tiny inputs)
# --------------------------------------------------------------------------

def dataspace_matrix(G, cov, lam) -> np.ndarray:
    """A = G C G^T + lambda I (the N x N system of Eq. 10-11)."""
    return G @ (cov[:, None] * G.T) + lam * np.eye(G.shape[0])


def invert_dense(G, cov, lam, d_obs, m_ref=None):
    """Eq. 11 with a Cholesky solve: y = A^-1 delta_d, m = m_ref + C G^T y."""
    m_ref = np.zeros(G.shape[1]) if m_ref is None else np.asarray(m_ref, dtype=np.float64)
    dd = d_obs - G @ m_ref
    A = dataspace_matrix(G, cov, lam)
    y = cho_solve(cho_factor(A), dd)
    return m_ref + cov * (G.T @ y), y


def invert_model_space(G, cov, lam, d_obs, m_ref=None):
    """Eq. 8 solved directly (M x M; tiny inputs only):
    (G^T W_d^-1 G + W_m^-1) (m - m_ref) = G^T W_d^-1 (d_obs - G m_ref)."""
    m_ref = np.zeros(G.shape[1]) if m_ref is None else np.asarray(m_ref, dtype=np.float64)
    dd = d_obs - G @ m_ref
    H = G.T @ G / lam + np.diag(1.0 / cov)
    rhs = G.T @ dd / lam
    return m_ref + cho_solve(cho_factor(H), rhs)


# --------------------------------------------------------------------------
# Matrix-free forms
# --------------------------------------------------------------------------

def dataspace_apply(mesh, obs, wdepth, lam, v) -> np.ndarray:
    """A v = G C G^T v + lambda v, matrix-free."""
    cov = covariance_from_weights(wdepth)
    return prism.forward(mesh, obs, cov * prism.adjoint(mesh, obs, v)) + lam * np.asarray(v)


def conjugate_gradient(apply, b, tol=0.0, max_iter=100, fixed_iters=None, y0=None):
    """Plain conjugate gradients on the SPD system A y = b from y0 (default 0).

    Stops when ||b - A y|| / ||b|| <= tol (recursively updated residual) or
    after max_iter iterations; ``fixed_iters`` runs exactly that many.
    Returns (y, iterations, relres_history), the history starting with the
    relative residual of y0."""
    b = np.asarray(b, dtype=np.float64)
    y = np.zeros_like(b) if y0 is None else np.array(y0, dtype=np.float64)
    r = b.copy() if y0 is None else b - apply(y)
    p = r.copy()
    rr = float(r @ r)
    bnorm = np.linalg.norm(b)
    hist = [np.sqrt(rr) / bnorm]
    if fixed_iters is None and hist[0] <= tol:
        return y, 0, hist
    n_iter = fixed_iters if fixed_iters is not None else max_iter
    it = 0
    for it in range(1, n_iter + 1):
        q = apply(p)
        alpha = rr / float(p @ q)
        y += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        hist.append(np.sqrt(rr_new) / bnorm)
        if fixed_iters is None and hist[-1] <= tol:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return y, it, hist


def invert_cg(mesh, obs, d_obs, wdepth, lam, m_ref=None, tol=1e-6, max_iter=200,
              fixed_iters=None):
    """Data-space inversion with matrix-free CG (Eq. 11): returns
    (m, y, iterations, relres_history)."""
    cov = covariance_from_weights(wdepth)
    m_ref = np.zeros(mesh.ncells) if m_ref is None else np.asarray(m_ref, dtype=np.float64)
    dd = np.asarray(d_obs, dtype=np.float64) - prism.forward(mesh, obs, m_ref)
    y, it, hist = conjugate_gradient(
        lambda p: dataspace_apply(mesh, obs, wdepth, lam, p), dd, tol=tol,
        max_iter=max_iter, fixed_iters=fixed_iters)
    m = m_ref + cov * prism.adjoint(mesh, obs, y)
    return m, y, it, hist


def restarted_cg(apply, b, inner=20, outer=30, tol=1e-4, max_halvings=5, log=None, y0=None):
    """The paper's solver policy (Section 2.2: at most `outer` model updates,
    each at most `inner` CG iterations, stop at res <= tol, step-size
    backtracking), in the reading used here:

    * outer cycle: restart CG from the current y with the true residual
      r = b - A y and p = r; run up to `inner` iterations (stop early when
      ||r|| / ||b|| <= tol);
    * backtracking: Q(y) = y^T A y / 2 - y^T b = -(y^T (b + r)) / 2 is the
      quadratic the data-space system minimises; while the cycle raised Q,
      halve its step (y <- y_old + (y - y_old) / 2, r recomputed), at most
      `max_halvings` times;
    * stop when ||r|| / ||b|| <= tol after a cycle, or after `outer` cycles.

    If ``log`` is a list, the recursive relative residual after every inner
    iteration is appended to it (the misfit-versus-iteration record).  ``y0``
    starts from that iterate instead of 0 (residuals stay relative to ||b||).

    Returns (y, total_inner_iterations, outer_cycles, relres_history), the
    history holding the true relative residual after each cycle."""
    b = np.asarray(b, dtype=np.float64)
    y = np.zeros_like(b) if y0 is None else np.array(y0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    r = b - apply(y)
    hist = [float(np.linalg.norm(r)) / bnorm]
    total = 0
    q_old = -0.5 * float(y @ (b + r))     # Q(y0); 0 for y0 = 0
    cycles = 0
    if hist[0] <= tol:
        return y, 0, 0, hist
    for cycles in range(1, outer + 1):
        y_old = y.copy()
        r = b - apply(y)
        p = r.copy()
        rr = float(r @ r)
        for _ in range(inner):
            if np.sqrt(rr) / bnorm <= tol:
                break
            q = apply(p)
            alpha = rr / float(p @ q)
            y = y + alpha * p
            r = r - alpha * q
            rr_new = float(r @ r)
            p = r + (rr_new / rr) * p
            rr = rr_new
            total += 1
            if log is not None:
                log.append(np.sqrt(rr) / bnorm)
        r = b - apply(y)
        q_new = -0.5 * float(y @ (b + r))
        halvings = 0
        while q_new > q_old and halvings < max_halvings:
            y = y_old + 0.5 * (y - y_old)
            r = b - apply(y)
            q_new = -0.5 * float(y @ (b + r))
            halvings += 1
        q_old = q_new
        hist.append(float(np.linalg.norm(r)) / bnorm)
        if hist[-1] <= tol:
            break
    return y, total, cycles, hist
