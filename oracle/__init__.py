"""Plain FP64 CPU oracle for the prism-gravity operators and the data-space
inversion.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product library never does, and the two
share no code.  Every function cites the equation it follows (paper Eq. 1-11).

Parity status of each function (what pins it, besides itself):

* ``prism.psi`` / ``prism.prism_corner_sum``: Bouguer-slab limit, cube
  far-field (point-mass) limit, voxel sphere vs analytic sphere,
  sub-prism superposition, mirror symmetry, reflection sign flip, 50-digit
  mpmath evaluation of the literal Eq. 1-3.
* ``prism.forward`` / ``adjoint`` / ``sensitivity_row`` /
  ``weighted_row_sumsq`` / ``forward_multi``: equal to the literal per-prism
  form on small meshes; single-cell index-order check.
* ``inversion.invert_dense`` / ``invert_model_space``: Eq. 9 identity (the two
  solves agree), normal-equation residual of Eq. 8.
* ``inversion.conjugate_gradient`` / ``invert_cg``: converge to the Cholesky
  solution.
* ``inversion.add_noise``: relative RMS of the added noise; R^2 consistency
  with the paper's two quoted values is a weak check only.
"""
from . import prism, inversion  # noqa: F401
from .prism import GAMMA  # noqa: F401
