"""The pins catch plausible mistakes.  Each test plants one mistake in the
oracle (on the CPU, by monkeypatching one of its step functions), runs the
pin meant to catch it, and checks that the pin now fails.  Nothing here
touches the GPU path."""

import numpy as np
import pytest
from scipy import stats

import oracle.linalg as OL
import oracle.philox as OP
import oracle.rsvd as OR
from paper_2402_17794_amd import workloads as W


def _sin_theta(Q1, Q2):
    return float(np.linalg.norm(Q2 - Q1 @ (Q1.T @ Q2), 2))


def _eq32_pin_error(q):
    """The eq. (3.2) range pin of test_oracle_rsvd on a square matrix
    (square so that a transposed operand still has matching shapes)."""
    n, l = 80, 12
    sig = W.spectrum_geometric(n, 0.9)
    U, V = W.haar(n, n, 21), W.haar(n, n, 22)
    A = (U * sig) @ V.T
    out = OR.rsvd_alg4(A, k=l, p=0, q=q, seed=4)
    Qref, _ = np.linalg.qr((U * sig ** (2 * q + 1)) @ (V.T @ OP.omega(4, n, l)))
    return _sin_theta(out["Q"], Qref)


def _exact_svd_pin_error():
    """The l = min(m, n) special case of test_oracle_rsvd: singular values and
    leading vectors against LAPACK."""
    sig = W.spectrum_geometric(40, 0.8)
    A = W.known_spectrum(40, 40, sig, 1, 2)       # square: a transposed operand still fits
    out = OR.rsvd_alg4(A, k=40, p=0, q=0, seed=1)
    Ul, _, Vtl = np.linalg.svd(A, full_matrices=False)
    err = np.max(np.abs(out["S"] - sig)) / sig[0]
    for i in range(5):
        s = np.sign(out["U"][:, i] @ Ul[:, i]) or 1.0
        err = max(err, np.max(np.abs(out["U"][:, i] - s * Ul[:, i])),
                  np.max(np.abs(out["Vt"][i] - s * Vtl[i])))
    return err


def test_pins_pass_unmutated():
    assert _eq32_pin_error(1) <= 1e-8
    assert _exact_svd_pin_error() <= 1e-9


def test_dropped_power_iteration_is_caught(monkeypatch):
    monkeypatch.setattr(OR, "_power_step", lambda A, Q: Q)
    assert _eq32_pin_error(1) > 1e-3


def test_transposed_operand_in_power_step_is_caught(monkeypatch):
    monkeypatch.setattr(OR, "_power_step", lambda A, Q: OR.orth(A @ OR.orth(A @ Q)))
    assert _eq32_pin_error(1) > 1e-3


def test_transposed_projection_is_caught(monkeypatch):
    monkeypatch.setattr(OR, "_project", lambda A, Q: Q.T @ A.T)
    assert _exact_svd_pin_error() > 1e-3


def test_wrong_lift_factor_is_caught(monkeypatch):
    # U = Q V-factor instead of Q U~
    orig = OL.jacobi_svd

    def swapped(X, **kw):
        Usv, s, J, c, sw = orig(X, **kw)
        return Usv, s, np.eye(J.shape[0]), c, sw
    monkeypatch.setattr(OR, "jacobi_svd", swapped)
    assert _exact_svd_pin_error() > 1e-3


def test_wrong_rotation_sign_is_caught(monkeypatch):
    orig = OL._rotation
    monkeypatch.setattr(OL, "_rotation", lambda a, b, g: (orig(a, b, g)[0], -orig(a, b, g)[1]))
    X = np.random.default_rng(3).standard_normal((30, 8))
    _, s, _, conv, _ = OL.jacobi_svd(X, max_sweeps=20)
    ref = np.linalg.svd(X, compute_uv=False)
    assert (not conv) or np.max(np.abs(s - ref)) > 1e-8


def test_missing_householder_sign_fix_is_caught(monkeypatch):
    monkeypatch.setattr(OL, "_positive_diagonal", lambda Q, R: (Q, R))
    Y = np.random.default_rng(4).standard_normal((50, 6))
    Q, R = OL.householder_qr(Y)
    Ql, Rl = np.linalg.qr(Y)
    d = np.where(np.diag(Rl) < 0, -1.0, 1.0)
    assert np.max(np.abs(Q - Ql * d)) > 1e-3 or np.any(np.diag(R) < 0)


def test_same_branch_box_muller_is_caught(monkeypatch):
    """Taking the cosine branch for both rows of a pair makes the even and
    odd rows identical: the row-independence part of the normality pin fails."""
    def bad(u1, u2):
        r = np.sqrt(-2.0 * np.log(u1))
        return r * np.cos(2 * np.pi * u2), r * np.cos(2 * np.pi * u2)
    monkeypatch.setattr(OP, "box_muller", bad)
    Om = OP.omega(0, 4000, 20)
    r = np.corrcoef(Om[0::2].ravel(), Om[1::2].ravel())[0, 1]
    assert abs(r) > 0.5


def test_log_of_wrong_uniform_is_caught(monkeypatch):
    """Feeding the [0, 1) uniform to the logarithm produces infinities at
    u = 0 and a biased radius: the moment / KS pin fails."""
    def bad(u1, u2):
        r = np.sqrt(-2.0 * np.log(np.maximum(1.0 - u2, 2.0 ** -24) ** 0.5))
        return r * np.cos(2 * np.pi * u1), r * np.sin(2 * np.pi * u1)
    monkeypatch.setattr(OP, "box_muller", bad)
    z = OP.omega(0, 20000, 50).ravel()
    assert stats.kstest(z, "norm").pvalue < 1e-6
