"""Thin Householder QR and one-sided (Hestenes) Jacobi SVD in float64.

Test infrastructure only (see the package docstring).

orth(Y).  Algorithms 1-4 ask for "a matrix whose columns form an orthonormal
basis for the range of Y" without naming a method.  The reading used here is
the thin QR factorisation Y = QR with no rank truncation (Q keeps all l
columns) and diag(R) >= 0, computed by Householder reflections.  For a
full-rank Y this Q is unique, so any correct orthonormalisation with a
non-negative triangular factor must agree with it up to rounding.

svd(B).  Stage 2 of Algorithms 2-4 computes "an SVD of the small matrix" with
a standard dense method.  The method used here is the one-sided Jacobi
(Hestenes) iteration: plane rotations applied on the right of X until its
columns are mutually orthogonal; then the column norms are the singular
values, the normalised columns the left singular vectors of X, and the
accumulated rotation the right singular vectors.
"""

import numpy as np


def householder_qr(Y):
    """Thin QR of an m x l matrix Y (m >= l): returns (Q m x l, R l x l) with
    Q^T Q = I, Y = Q R, R upper triangular and R_jj >= 0.

    Column j: reflect the trailing part x = R[j:, j] onto -sign(x_0)|x| e_1
    (the sign choice that avoids cancellation), apply the reflector to the
    trailing columns, and keep it.  Q is formed by applying the reflectors,
    last to first, to the first l columns of the identity.  A zero trailing
    column gets no reflector (R_jj = 0, Q's column j stays a unit vector
    orthogonal to the others).  Finally each column of Q whose R_jj is
    negative is negated together with row j of R.
    """
    Y = np.array(Y, dtype=np.float64, copy=True)
    m, l = Y.shape
    if l > m:
        raise ValueError("householder_qr needs rows >= cols")
    R = Y
    reflectors = []
    for j in range(l):
        x = R[j:, j].copy()
        normx = np.sqrt(np.dot(x, x))
        if normx == 0.0:
            reflectors.append(None)
            continue
        alpha = -normx if x[0] >= 0 else normx
        v = x
        v[0] -= alpha
        v /= np.sqrt(np.dot(v, v))
        R[j:, j:] -= 2.0 * np.outer(v, v @ R[j:, j:])
        reflectors.append(v)
    Q = np.zeros((m, l))
    Q[:l, :l] = np.eye(l)
    for j in range(l - 1, -1, -1):
        v = reflectors[j]
        if v is None:
            continue
        Q[j:, :] -= 2.0 * np.outer(v, v @ Q[j:, :])
    return _positive_diagonal(Q, np.triu(R[:l, :]))


def _positive_diagonal(Q, R):
    """Negate column j of Q and row j of R wherever R_jj < 0."""
    d = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return Q * d[None, :], R * d[:, None]


def _rotation(a, b, g):
    """Cosine and sine of the plane rotation that makes columns with squared
    norms a, b and inner product g orthogonal (the smaller of the two
    rotation angles)."""
    zeta = (b - a) / (2.0 * g)
    t = (1.0 if zeta >= 0 else -1.0) / (abs(zeta) + np.hypot(1.0, zeta))
    c = 1.0 / np.sqrt(1.0 + t * t)
    return c, c * t


def orth(Y):
    """Orthonormal basis of range(Y) with exactly Y.shape[1] columns."""
    return householder_qr(Y)[0]


def jacobi_svd(X, tol=1e-15, max_sweeps=60):
    """One-sided Jacobi SVD of a rows x l matrix X (rows >= l).

    Cyclic-by-row sweeps over column pairs (i < j).  With a = |x_i|^2,
    b = |x_j|^2, g = x_i . x_j, a pair is left alone when
    |g| <= tol * sqrt(a b); otherwise zeta = (b - a) / (2 g),
    t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) (sign(0) = +1),
    c = 1 / sqrt(1 + t^2), s = c t, and columns i, j of X and of the
    accumulated rotation J become (c x_i - s x_j, s x_i + c x_j), which makes
    them orthogonal.  Iteration stops after a sweep without rotations, or
    after max_sweeps sweeps (then converged = False).

    Returns (Usv, sigma, J, converged, sweeps) with X J = Usv diag(sigma),
    sigma sorted descending (stable by column index), Usv the normalised
    columns (a zero column stays zero) and J orthogonal.
    """
    X = np.array(X, dtype=np.float64, copy=True)
    rows, l = X.shape
    Xt = np.ascontiguousarray(X.T)       # Xt[i] is column i of X
    Jt = np.eye(l)                       # Jt[i] is column i of J
    converged = False
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        rotated = False
        for i in range(l - 1):
            for j in range(i + 1, l):
                xi, xj = Xt[i], Xt[j]
                a = np.dot(xi, xi)
                b = np.dot(xj, xj)
                g = np.dot(xi, xj)
                if abs(g) <= tol * np.sqrt(a * b):
                    continue
                c, s = _rotation(a, b, g)
                Xt[i], Xt[j] = c * xi - s * xj, s * xi + c * xj
                ji, jj = Jt[i].copy(), Jt[j].copy()
                Jt[i], Jt[j] = c * ji - s * jj, s * ji + c * jj
                rotated = True
        if not rotated:
            converged = True
            break
    sigma = np.sqrt(np.einsum("ij,ij->i", Xt, Xt))
    order = np.argsort(-sigma, kind="stable")
    Usv = np.zeros((rows, l))
    nz = sigma > 0
    Usv[:, nz] = (Xt[nz] / sigma[nz, None]).T
    return Usv[:, order], sigma[order], Jt.T[:, order], converged, sweeps
