"""FP64 CPU oracle for the randomized SVD hot path (test infrastructure only).

This package is the plain, slow reference that the GPU library is checked
against.  It is TEST INFRASTRUCTURE: only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The product path (the
HIP library and its Python binding) never imports, links or calls anything in
here, and this package imports nothing from the product.

Modules
  philox   counter-based Philox4xW-R generator and the Box-Muller Gaussian
           test matrix (Algorithm 4 step 1: the Gaussian test matrix).
  linalg   thin Householder QR (the "orth" of Algorithms 1-4) and the
           one-sided Jacobi SVD (the "standard algorithm" of Stage 2).
  rsvd     Algorithm 4 end to end (Algorithm 2 is q = 0), the residual
           norms of the error measure, Algorithm 3 for comparison.
  bounds   the expected-error bounds of Theorems 2, 3, 6 and eq. (3.5), the
           canonical-angle bounds of Theorem 5, and the Eckart-Young floor
           of eq. (3.1).
  angles   canonical angles between subspaces (Section 4.3).
  adaptive the adaptive randomized range finder (Appendix A, blocked).
  srft     the SRFT test matrix and FastRandRF (Appendix A).
  single_pass  the single-pass Algorithms 5 (Hermitian) and 6 (general) of
           Section 3.4.

Everything is real (the paper's conjugate transpose becomes a transpose) and
computed in float64.
"""

from . import philox, linalg, rsvd, bounds, quant, angles, adaptive, srft, single_pass  # noqa: F401
from .rsvd import rsvd_alg4, rsvd_alg3, residual_norms  # noqa: F401
