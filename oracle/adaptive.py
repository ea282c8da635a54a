"""Adaptive randomized range finder (Appendix A, Adaptive_randRF: given A,
a tolerance eps and an integer r, an orthonormal Q with ||(I - Q Q^T) A|| <=
eps with probability at least 1 - min(m, n) 10^-r).  Test infrastructure
only (see the package docstring).

The reading used here is the blocked form of that algorithm, with blocks of
b = r Gaussian vectors, which is what a GPU can run (one skinny product per
block), and a rank-revealing append, so that a block that is numerically
rank-deficient (an exact-rank A, or a block straddling the numerical rank)
adds only the directions it really holds:

  Q = [] (m x 0); t = 0
  repeat
    Omega_t = columns t b .. t b + b - 1 of the Gaussian test matrix on
              Philox stream 3 (oracle.philox.omega with stream 3)
    Y = A Omega_t;  Y = Y - Q (Q^T Y), done twice
    est = 10 sqrt(2 / pi) max_i ||Y e_i||
    if est <= eps: stop (converged)
    Y = W S Z^T (thin SVD); keep the s columns of W with S_ii > eps / (10 sqrt(2/pi))
    (s >= 1: S_11 >= max_i ||Y e_i||)
    if Q would exceed max_l columns: stop (not converged)
    W_s = W_s - Q (Q^T W_s);  Q = [Q, orth(W_s)]
    t = t + 1

The stopping test is the a-posteriori bound the algorithm rests on: for a
matrix B and b independent standard Gaussian vectors, ||B|| <= 10 sqrt(2/pi)
max_i ||B w_i|| except with probability 10^-b; applied to B = (I - Q Q^T) A.
The directions left out of a block have singular values below eps / (10
sqrt(2/pi)); if they matter, later blocks sample them again.
"""

import math

import numpy as np

from .linalg import orth
from .philox import omega

ADAPTIVE_STREAM = 3
EST_FACTOR = 10.0 * math.sqrt(2.0 / math.pi)


def _project(Q, Y):
    return Y - Q @ (Q.T @ Y) if Q.shape[1] else Y


def adaptive_range_finder(A, tol, block=16, max_l=None, seed=0):
    """Returns dict(Q (m x l), l, est, converged, blocks)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    b = int(block)
    if b < 1 or tol < 0:
        raise ValueError("need block >= 1 and tol >= 0")
    cap = min(m, n) if max_l is None else min(int(max_l), min(m, n))
    Q = np.zeros((m, 0))
    t = 0
    while True:
        Om = omega(seed, n, (t + 1) * b, stream=ADAPTIVE_STREAM)[:, t * b:]
        Y = _project(Q, _project(Q, A @ Om))
        est = EST_FACTOR * float(np.max(np.linalg.norm(Y, axis=0)))
        if est <= tol:
            return dict(Q=Q, l=Q.shape[1], est=est, converged=True, blocks=t + 1)
        Wl, S, _ = np.linalg.svd(Y, full_matrices=False)
        keep = int(np.sum(S > tol / EST_FACTOR))
        if Q.shape[1] + keep > cap:
            return dict(Q=Q, l=Q.shape[1], est=est, converged=False, blocks=t + 1)
        Q = np.concatenate([Q, orth(_project(Q, Wl[:, :keep]))], axis=1)
        t += 1


__all__ = ["adaptive_range_finder", "ADAPTIVE_STREAM", "EST_FACTOR"]
