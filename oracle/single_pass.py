"""Single-pass randomized factorizations (Section 3.4) in float64.

Test infrastructure only (see the package docstring).

Both methods touch every entry of A once: all products with A are sketches
formed from the same read of A, and Stage 2 works only on the sketches.

Algorithm 5 (Section 3.4.1, Hermitian A, n x n, l = k + p):
  1-3  Omega: n x l Gaussian test matrix (stream 0); Y = A Omega; Q = orth(Y)
  4    C solves C (Q^T Omega) = Q^T Y          (eq. (3.13))
  5    eigendecomposition C = U^ D U^T
  6    U = Q U^

Algorithm 6 (Section 3.4.2, general A, m x n, l = k + p):
  1-2  Omega_c: n x l (stream 0), Omega_r: m x l (stream 1);
       Y_c = A Omega_c, Y_r = A^T Omega_r
  3    Q_c, Q_r: the k dominant left singular vectors of Y_c, Y_r
  4    C (k x k) is the least-squares solution of the joint system
       (Omega_r^T Q_c) C = Y_r^T Q_r  and  C (Q_r^T Omega_c) = Q_c^T Y_c
  5    C = U^ Sigma V^^T
  6    U = Q_c U^, V = Q_r V^

Readings taken where the text is silent or garbled:
  * Algorithm 5: C is l x l (Q has l columns; the k x k of the listing is
    read as a slip).  C is the solution of the square system, computed by LU
    with partial pivoting.  With rounding, and whenever A is not exactly of
    rank <= l, C is not symmetric; step 5 takes the eigendecomposition of its
    symmetric part (C + C^T) / 2, the nearest symmetric matrix.  The rank-k
    result keeps the k eigenvalues of largest magnitude (A may be
    indefinite), ordered by |lambda| descending and, on a tie, by lambda
    descending.  Each eigenvector's entry of largest magnitude (lowest index
    on ties) is made positive.
  * Algorithm 6: Y_r = A^T Omega_r (Omega_r has m rows; the listing's
    A Omega_r is read as a slip).  Step 3 keeps k columns, so each of the two
    equations is overdetermined (l x k and k x l); the joint least-squares
    problem minimises ||M1 C - N1||_F^2 + ||C M2 - N2||_F^2 with equal
    weights, whose minimiser solves the Sylvester equation
    (M1^T M1) C + C (M2 M2^T) = M1^T N1 + N2 M2^T  (both coefficient
    matrices are positive definite when M1, M2^T have full column rank).
    The small SVD and the sign rule are those of Algorithm 4.
"""

import numpy as np
import scipy.linalg

from .linalg import jacobi_svd, orth
from .philox import omega as gaussian_omega


def _sign_columns(X):
    """Make each column's entry of largest magnitude (lowest index on ties)
    positive; returns the signs applied."""
    sgn = np.ones(X.shape[1])
    for i in range(X.shape[1]):
        idx = int(np.argmax(np.abs(X[:, i])))
        if X[idx, i] < 0:
            sgn[i] = -1.0
    return sgn


def solve_right(W, Z):
    """C with C W = Z for a square, nonsingular W (eq. (3.13)): LU with
    partial pivoting on the transposed system W^T C^T = Z^T."""
    return np.linalg.solve(np.asarray(W, dtype=np.float64).T, np.asarray(Z, dtype=np.float64).T).T


def joint_lstsq(M1, N1, M2, N2):
    """Least-squares C (k x k) of the joint system M1 C = N1 (M1, N1: l x k)
    and C M2 = N2 (M2, N2: k x l), equal weights: the solution of the
    normal equations P C + C S = F with P = M1^T M1, S = M2 M2^T and
    F = M1^T N1 + N2 M2^T, by the Bartels-Stewart method."""
    M1, N1, M2, N2 = (np.asarray(x, dtype=np.float64) for x in (M1, N1, M2, N2))
    P = M1.T @ M1
    S = M2 @ M2.T
    F = M1.T @ N1 + N2 @ M2.T
    return scipy.linalg.solve_sylvester(P, S, F)


def dominant_left_singular(Y, k):
    """The k dominant left singular vectors of Y (columns of an orthonormal
    rows x k matrix), from a library SVD."""
    U, _, _ = np.linalg.svd(np.asarray(Y, dtype=np.float64), full_matrices=False)
    return U[:, :k].copy()


def two_sided_sketch(A, Oc, Or):
    """Step 2 of Algorithm 6: Y_c = A Omega_c and Y_r = A^T Omega_r, both
    formed from the same read of A."""
    return A @ Oc, A.T @ Or


def symmetric_part(C):
    """(C + C^T) / 2."""
    return 0.5 * (C + C.T)


def rsvd_alg5(A, k, p=10, seed=0, omega=None):
    """Algorithm 5 for a symmetric n x n A.  Returns a dict with U (n x k),
    D (k eigenvalues, |D| descending), the solved C (l x l, before
    symmetrisation), Q (n x l), l and Omega."""
    A = np.asarray(A, dtype=np.float64)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("Algorithm 5 needs a square (Hermitian) matrix")
    n = A.shape[0]
    k, p = int(k), int(p)
    if not (1 <= k <= n) or p < 0:
        raise ValueError("need 1 <= k <= n, p >= 0")
    l = min(k + p, n)
    Om = gaussian_omega(seed, n, l) if omega is None else np.asarray(omega, dtype=np.float64)
    if Om.shape != (n, l):
        raise ValueError("omega must be n x l")
    Y = A @ Om                                   # step 2: the one pass over A
    Q = orth(Y)                                  # step 3
    C = solve_right(Q.T @ Om, Q.T @ Y)           # step 4
    lam, Uh = np.linalg.eigh(symmetric_part(C))  # step 5
    order = np.lexsort((-lam, -np.abs(lam)))[:k]
    lam, Uh = lam[order], Uh[:, order]
    U = Q @ Uh                                   # step 6
    U = U * _sign_columns(U)[None, :]
    return dict(U=U, D=lam.copy(), C=C, Q=Q, l=l, omega=Om)


def rsvd_alg6(A, k, p=10, seed=0, omega_c=None, omega_r=None):
    """Algorithm 6 for an m x n A.  Returns a dict with U (m x k), S (k),
    Vt (k x n), C (k x k), Q_c (m x k), Q_r (n x k), l, and the two test
    matrices."""
    A = np.asarray(A, dtype=np.float64)
    if A.ndim != 2:
        raise ValueError("A must be a matrix")
    m, n = A.shape
    k, p = int(k), int(p)
    if not (1 <= k <= min(m, n)) or p < 0:
        raise ValueError("need 1 <= k <= min(m, n), p >= 0")
    l = min(k + p, min(m, n))
    Oc = gaussian_omega(seed, n, l, stream=0) if omega_c is None else np.asarray(omega_c, dtype=np.float64)
    Or = gaussian_omega(seed, m, l, stream=1) if omega_r is None else np.asarray(omega_r, dtype=np.float64)
    if Oc.shape != (n, l) or Or.shape != (m, l):
        raise ValueError("omega_c must be n x l and omega_r m x l")
    Yc, Yr = two_sided_sketch(A, Oc, Or)         # step 2 (both sketches from one pass)
    Qc = dominant_left_singular(Yc, k)           # step 3
    Qr = dominant_left_singular(Yr, k)
    C = joint_lstsq(Or.T @ Qc, Yr.T @ Qr,        # step 4
                    Qr.T @ Oc, Qc.T @ Yc)
    Vsv, sig, J, conv, _ = jacobi_svd(C.T)       # step 5: C = J Sigma Vsv^T
    U = Qc @ J                                   # step 6
    V = Qr @ Vsv
    sgn = _sign_columns(V)
    U, V = U * sgn[None, :], V * sgn[None, :]
    return dict(U=U, S=sig.copy(), Vt=V.T.copy(), C=C, Q_c=Qc, Q_r=Qr, l=l, omega_c=Oc, omega_r=Or,
                converged=conv)


__all__ = ["rsvd_alg5", "rsvd_alg6", "joint_lstsq", "solve_right", "dominant_left_singular",
           "two_sided_sketch", "symmetric_part"]
