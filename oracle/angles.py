"""Canonical angles between subspaces (Section 4.3, eq. (4.3), and the
angles of Theorem 5).  Test infrastructure only (see the package docstring).

For U1 (m x k) and U2 (m x l) with orthonormal columns and k <= l, the
canonical angles theta_1 <= ... <= theta_k between range(U1) and range(U2)
have cosines the singular values of U1^T U2 and sines the singular values of
(I - U2 U2^T) U1.  The sines are computed from the latter (accurate for
small angles), with a library SVD as a step, and returned in ascending
order.
"""

import numpy as np


def canonical_sines(U1, U2):
    """sin theta_1 <= ... <= sin theta_k for range(U1) against range(U2)."""
    U1 = np.asarray(U1, dtype=np.float64)
    U2 = np.asarray(U2, dtype=np.float64)
    if U1.shape[1] > U2.shape[1]:
        raise ValueError("need k <= l")
    E = U1 - U2 @ (U2.T @ U1)
    s = np.linalg.svd(E, compute_uv=False) if E.size else np.zeros(0)
    return np.sort(np.minimum(s, 1.0))


def canonical_cosines(U1, U2):
    """cos theta_1 >= ... >= cos theta_k (singular values of U1^T U2)."""
    return np.sort(np.minimum(np.linalg.svd(np.asarray(U1).T @ np.asarray(U2), compute_uv=False), 1.0))[::-1]


__all__ = ["canonical_sines", "canonical_cosines"]
