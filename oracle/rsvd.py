"""Algorithm 4 (randomized SVD with re-orthonormalised power iterations) in
float64, step by step, plus the error measure.  Test infrastructure only.

Algorithm 4 (Chapter 3, Section 3.3), for an m x n matrix A, target rank k,
oversampling p and power exponent q, with l = k + p:

  Stage 1
    1  Omega: n x l Gaussian test matrix
    2  Y = A Omega
    3  Q = orth(Y)
    4-5  repeat q times:  W = orth(A^T Q);  Q = orth(A W)
  Stage 2
    6  B = Q^T A
    7  B = U~ Sigma V^T  (SVD of the small l x n matrix)
    8  U = Q U~

Algorithm 2 (Section 3.1) is the q = 0 case.  Readings taken where the paper
is silent:
  * l = min(k + p, min(m, n)) (the image experiments run k + p past min(m, n));
    1 <= k <= min(m, n), p >= 0, q >= 0 are required.
  * orth is the thin Householder QR with diag(R) >= 0 (oracle.linalg).
  * The small SVD is the one-sided Jacobi iteration applied to X = B^T:
    B^T J = Usv Sigma gives B = J Sigma Usv^T, so U~ = J and V = Usv.
  * The paper returns a rank-(k+p) factorisation and mentions truncating the
    last p components; by default the top k are returned.
  * Signs: for each returned singular pair, the entry of largest magnitude in
    the column of V (lowest row index on ties) is made positive, negating the
    matching column of U.
"""

import numpy as np

from .linalg import householder_qr, jacobi_svd, orth
from .philox import omega as gaussian_omega


def _validate(A, k, p, q):
    A = np.asarray(A, dtype=np.float64)
    if A.ndim != 2:
        raise ValueError("A must be a matrix")
    m, n = A.shape
    k, p, q = int(k), int(p), int(q)
    if not (1 <= k <= min(m, n)) or p < 0 or q < 0:
        raise ValueError("need 1 <= k <= min(m, n), p >= 0, q >= 0")
    return A, m, n, k, p, q, min(k + p, min(m, n))


def _sketch(A, Om):
    """Step 2: Y = A Omega."""
    return A @ Om


def _power_step(A, Q):
    """One pass of the loop of steps 4-5: W = orth(A^T Q); Q = orth(A W)."""
    W = orth(A.T @ Q)
    return orth(A @ W)


def _project(A, Q):
    """Step 6: B = Q^T A."""
    return Q.T @ A


def _lift(Q, Ut):
    """Step 8: U = Q U~."""
    return Q @ Ut


def _stage2(A, Q, k, l, return_full_l):
    """Steps 6-8 and the truncation/sign conventions."""
    B = _project(A, Q)                                   # step 6
    Usv, sig, J, conv, sweeps = jacobi_svd(B.T)          # step 7 on X = B^T
    U = _lift(Q, J)                                      # step 8 (U~ = J)
    r = l if return_full_l else k
    U, S, V = U[:, :r].copy(), sig[:r].copy(), Usv[:, :r].copy()
    for i in range(r):
        idx = int(np.argmax(np.abs(V[:, i])))
        if V[idx, i] < 0:
            V[:, i] = -V[:, i]
            U[:, i] = -U[:, i]
    return dict(U=U, S=S, Vt=V.T.copy(), B=B, converged=conv, sweeps=sweeps)


def rsvd_alg4(A, k, p=10, q=0, seed=0, omega=None, return_full_l=False):
    """Algorithm 4.  Returns a dict with U (m x r), S (r), Vt (r x n), the
    final Q (m x l), B = Q^T A (l x n), l, and the Jacobi convergence flag,
    where r = k, or l with return_full_l.  `omega` replaces step 1 with a
    given n x l matrix."""
    A, m, n, k, p, q, l = _validate(A, k, p, q)
    Om = gaussian_omega(seed, n, l) if omega is None else np.asarray(omega, dtype=np.float64)
    if Om.shape != (n, l):
        raise ValueError("omega must be n x l")
    Y = _sketch(A, Om)                                   # step 2
    Q = orth(Y)                                          # step 3
    for _ in range(q):                                   # steps 4-5
        Q = _power_step(A, Q)
    out = _stage2(A, Q, k, l, return_full_l)
    out.update(Q=Q, l=l, omega=Om)
    return out


def rsvd_alg3(A, k, p=10, q=0, seed=0, omega=None, return_full_l=False):
    """Algorithm 3 (Section 3.2): the power scheme without orthonormalisation
    between products: Y = A Omega, then q times Z = A^T Y, Y = A Z, then
    Q = orth(Y) and the same Stage 2."""
    A, m, n, k, p, q, l = _validate(A, k, p, q)
    Om = gaussian_omega(seed, n, l) if omega is None else np.asarray(omega, dtype=np.float64)
    Y = A @ Om
    for _ in range(q):
        Z = A.T @ Y
        Y = A @ Z
    Q = orth(Y)
    out = _stage2(A, Q, k, l, return_full_l)
    out.update(Q=Q, l=l, omega=Om)
    return out


def spectral_norm_power(E, iters=30, block=16, seed=0):
    """Largest singular value of E by block power iteration on E^T E with a
    Gaussian start block (Philox stream 2), re-orthonormalised every
    half-step, then a Rayleigh-Ritz step: the largest singular value of
    E Z for the final orthonormal n x b block Z."""
    E = np.asarray(E, dtype=np.float64)
    m, n = E.shape
    b = min(block, n, m)
    Z = orth(gaussian_omega(seed, n, b, stream=2))
    for _ in range(iters):
        Y = orth(E @ Z)
        Z = orth(E.T @ Y)
    _, s, _, _, _ = jacobi_svd(E @ Z)
    return float(s[0])


def residual_norms(A, Q, exact_limit=1 << 22):
    """The error measure ||A - Q Q^T A|| of Theorems 2, 3, 6 (spectral norm)
    and its Frobenius counterpart, for the full l-column Q.  The spectral
    norm is exact (largest singular value by a library SVD) when
    m * n <= exact_limit, otherwise the block power estimate."""
    A = np.asarray(A, dtype=np.float64)
    E = A - Q @ (Q.T @ A)
    fro = float(np.sqrt(np.sum(E * E)))
    if E.size <= exact_limit:
        spec = float(np.linalg.svd(E, compute_uv=False)[0]) if E.size else 0.0
    else:
        spec = spectral_norm_power(E)
    return spec, fro


__all__ = ["rsvd_alg4", "rsvd_alg3", "residual_norms",
           "spectral_norm_power", "householder_qr", "jacobi_svd"]
