"""Pins for the oracle's Householder QR and one-sided Jacobi SVD.

Each is checked against what fixes it independently: LAPACK (numpy) QR and
SVD as library special cases, the closed-form singular values of a 2 x 2
matrix, and the defining identities (orthonormality, reconstruction,
triangularity, sign of diag(R)).
"""

import numpy as np
import pytest

from oracle.linalg import householder_qr, jacobi_svd


def _orth_err(Q):
    return np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1])))


@pytest.mark.parametrize("m,l", [(1, 1), (5, 5), (40, 7), (300, 30), (1000, 64)])
def test_householder_matches_lapack_qr(m, l):
    Y = np.random.default_rng(m + l).standard_normal((m, l))
    Q, R = householder_qr(Y)
    assert _orth_err(Q) <= 1e-12
    assert np.linalg.norm(Q @ R - Y) <= 1e-13 * np.linalg.norm(Y)
    assert np.allclose(R, np.triu(R)) and np.all(np.diag(R) >= 0)
    Ql, Rl = np.linalg.qr(Y)
    d = np.where(np.diag(Rl) < 0, -1.0, 1.0)
    assert np.max(np.abs(Q - Ql * d)) <= 1e-10
    assert np.max(np.abs(R - Rl * d[:, None])) <= 1e-10 * np.max(np.abs(R))


def test_householder_rank_deficient_and_zero():
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((200, 4)) @ rng.standard_normal((4, 12))   # rank 4, 12 columns
    Q, R = householder_qr(Y)
    assert _orth_err(Q) <= 1e-12
    assert np.linalg.norm(Q @ R - Y) <= 1e-13 * np.linalg.norm(Y)
    Qz, Rz = householder_qr(np.zeros((30, 5)))
    assert _orth_err(Qz) == 0.0 and np.all(Rz == 0.0)


def test_householder_ill_conditioned_orthonormal():
    rng = np.random.default_rng(2)
    U, _ = np.linalg.qr(rng.standard_normal((500, 20)))
    V, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    Y = (U * np.logspace(0, -12, 20)) @ V.T
    Q, R = householder_qr(Y)
    assert _orth_err(Q) <= 1e-12
    assert np.linalg.norm(Q @ R - Y) <= 1e-13 * np.linalg.norm(Y)


@pytest.mark.parametrize("rows,l", [(2, 2), (3, 3), (10, 4), (64, 64), (200, 30)])
def test_jacobi_matches_lapack_svd(rows, l):
    X = np.random.default_rng(rows * 7 + l).standard_normal((rows, l))
    Usv, s, J, conv, _ = jacobi_svd(X)
    assert conv
    s_ref = np.linalg.svd(X, compute_uv=False)
    assert np.max(np.abs(s - s_ref)) <= 1e-13 * s_ref[0]
    assert np.linalg.norm(X @ J - Usv * s) <= 1e-13 * np.linalg.norm(X)
    assert np.linalg.norm(X - (Usv * s) @ J.T) <= 1e-13 * np.linalg.norm(X)
    assert _orth_err(J) <= 1e-13 and _orth_err(Usv) <= 1e-13
    assert np.all(np.diff(s) <= 0)


@pytest.mark.parametrize("a,b,c,d", [(3.0, 1.0, -2.0, 5.0), (1.0, 0.0, 0.0, 1e-8),
                                     (0.0, 2.0, 2.0, 0.0), (1.0, 1.0, 1.0, 1.0)])
def test_jacobi_2x2_closed_form(a, b, c, d):
    X = np.array([[a, b], [c, d]])
    S = a * a + b * b + c * c + d * d
    D = abs(a * d - b * c)
    disc = np.sqrt(max(S * S - 4 * D * D, 0.0))
    s1 = np.sqrt((S + disc) / 2)
    s2 = 2 * D / np.sqrt(2 * (S + disc))            # = sqrt((S - disc)/2), cancellation-free
    _, s, _, conv, _ = jacobi_svd(X)
    assert conv
    assert s[0] == pytest.approx(s1, rel=1e-14)
    assert s[1] == pytest.approx(s2, rel=1e-12, abs=1e-15 * s1)


def test_jacobi_graded_and_rank_deficient():
    rng = np.random.default_rng(5)
    U, _ = np.linalg.qr(rng.standard_normal((80, 12)))
    V, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    sig = np.array([1.0, 0.5, 0.25, 1e-3, 1e-6, 1e-9, 0, 0, 0, 0, 0, 0])
    X = (U * sig) @ V.T
    Usv, s, J, conv, _ = jacobi_svd(X)
    assert conv
    assert np.max(np.abs(s - sig)) <= 1e-14
    assert _orth_err(J) <= 1e-13
    assert np.linalg.norm(X - (Usv * s) @ J.T) <= 1e-14


def test_jacobi_sweep_cap_reports_not_converged():
    X = np.random.default_rng(6).standard_normal((20, 10))
    _, _, _, conv, sweeps = jacobi_svd(X, max_sweeps=1)
    assert not conv and sweeps == 1
