"""FP64 CPU oracle for the regional-residual separation: least-squares
polynomial trend surface in the horizontal coordinates (the second-degree
trend removal of the field workflow, Section 2.2; one surface over the whole
domain joins separately inverted sections, Section 4.5).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

The fit is the plain definition: the polynomial of the given degree in (x, y)
that minimises sum_i (v_i - T(x_i, y_i))^2, solved with NumPy's SVD-based
least squares on the monomials of the coordinates taken relative to their
mean.  The fitted values T(x_i, y_i) do not depend on that choice of origin,
which is what parity is checked on.
"""
from __future__ import annotations

import numpy as np


def monomials(x, y, degree):
    """Columns x^a y^b with a + b <= degree."""
    cols = [x ** (d - b) * y ** b for d in range(degree + 1) for b in range(d + 1)]
    return np.stack(cols, axis=1)


def trend_surface(x, y, v, degree=2):
    """Returns (trend values T(x_i, y_i), residual v - T)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    X = monomials(x - x.mean(), y - y.mean(), degree)
    coef, *_ = np.linalg.lstsq(X, v, rcond=None)
    t = X @ coef
    return t, v - t
