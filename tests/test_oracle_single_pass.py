"""Pins for the oracle's single-pass Algorithms 5 and 6 (Section 3.4).

Nothing here compares the oracle with itself.  The pins are what the
mathematics fixes:
* the joint least-squares step of Algorithm 6 against brute force: the
  Kronecker form of the two equations solved by a library least-squares
  routine; a consistent system is solved exactly; with only the first
  equation the problem is an ordinary least-squares problem;
* the square solve of Algorithm 5 returns the matrix that generated its
  right-hand side;
* exact recovery: when A has rank <= l the sketches capture its range, so
  C equals the projection Q^T A Q of eq. (3.9) (Algorithm 5) or
  Q_c^T A Q_r of eq. (3.14) (Algorithm 6), and the returned eigen- or
  singular values and vectors are the generator's own;
* l = n (Algorithm 5) or k = l = min(m, n) (Algorithm 6): the methods
  become exact factorizations, checked against LAPACK;
* Eckart-Young (eq. (3.1)): no rank-k result beats sigma_{k+1};
* planted mistakes (a transposed operand in the second sketch, a sign in the
  normal equations) fail these pins.
"""

import numpy as np
import pytest

import oracle.single_pass as SP
from paper_2402_17794_amd import workloads as W


def _vec(X):
    return X.ravel(order="F")


def _kron_lstsq(M1, N1, M2, N2):
    """C minimising ||M1 C - N1||^2 + ||C M2 - N2||^2 by brute force:
    vec(M1 C) = (I kron M1) vec(C), vec(C M2) = (M2^T kron I) vec(C)."""
    k = M1.shape[1]
    I = np.eye(k)
    big = np.vstack([np.kron(I, M1), np.kron(M2.T, I)])
    rhs = np.concatenate([_vec(N1), _vec(N2)])
    x = np.linalg.lstsq(big, rhs, rcond=None)[0]
    return x.reshape(k, k, order="F")


@pytest.mark.parametrize("k,l,seed", [(1, 1, 0), (1, 4, 1), (3, 5, 2), (4, 4, 3), (6, 9, 4), (8, 20, 5)])
def test_joint_lstsq_matches_kronecker_brute_force(k, l, seed):
    rng = np.random.default_rng(seed)
    M1, N1 = rng.standard_normal((l, k)), rng.standard_normal((l, k))
    M2, N2 = rng.standard_normal((k, l)), rng.standard_normal((k, l))
    C = SP.joint_lstsq(M1, N1, M2, N2)
    ref = _kron_lstsq(M1, N1, M2, N2)
    assert np.max(np.abs(C - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))


def test_joint_lstsq_consistent_system_is_exact():
    rng = np.random.default_rng(7)
    k, l = 12, 17
    C0 = rng.standard_normal((k, k))
    M1, M2 = rng.standard_normal((l, k)), rng.standard_normal((k, l))
    C = SP.joint_lstsq(M1, M1 @ C0, M2, C0 @ M2)
    assert np.max(np.abs(C - C0)) <= 1e-11


def test_joint_lstsq_one_equation_is_ordinary_least_squares():
    rng = np.random.default_rng(8)
    k, l = 7, 15
    M1, N1 = rng.standard_normal((l, k)), rng.standard_normal((l, k))
    C = SP.joint_lstsq(M1, N1, np.zeros((k, l)), np.zeros((k, l)))
    ref = np.linalg.lstsq(M1, N1, rcond=None)[0]
    assert np.max(np.abs(C - ref)) <= 1e-11


def test_solve_right_returns_the_generating_matrix():
    rng = np.random.default_rng(9)
    l = 30
    C0, Wm = rng.standard_normal((l, l)), rng.standard_normal((l, l))
    assert np.max(np.abs(SP.solve_right(Wm, C0 @ Wm) - C0)) <= 1e-10


def _sym_exact_rank(n, r, seed=31):
    lam = np.zeros(n)
    lam[:r] = W.alternating_signs(0.8 ** np.arange(r))
    A = W.symmetric_spectrum(n, lam, seed)
    U = W.haar(n, n, seed)
    return A, lam, U


def _sign_fix(X):
    return X * np.where(X[np.argmax(np.abs(X), axis=0), np.arange(X.shape[1])] < 0, -1.0, 1.0)[None, :]


def test_alg5_exact_rank_recovers_the_eigendecomposition():
    n, r = 120, 12
    A, lam, U = _sym_exact_rank(n, r)
    out = SP.rsvd_alg5(A, k=r, p=8, seed=3)
    Q = out["Q"]
    # Eq. (3.9): with range(Y) = range(A), C is the projection Q^T A Q.
    assert np.max(np.abs(out["C"] - Q.T @ A @ Q)) <= 1e-11
    # Eigenvalues: the generator's, ordered by magnitude.
    order = np.argsort(-np.abs(lam[:r]), kind="stable")
    assert np.max(np.abs(out["D"] - lam[:r][order])) <= 1e-12
    # Eigenvectors: the generator's columns, with the sign rule.
    assert np.max(np.abs(out["U"] - _sign_fix(U[:, :r][:, order]))) <= 1e-10
    Ur = out["U"]
    assert np.max(np.abs(Ur.T @ Ur - np.eye(r))) <= 1e-12
    assert np.max(np.abs((Ur * out["D"]) @ Ur.T - A)) <= 1e-11


def test_alg5_full_width_is_an_exact_eigendecomposition():
    n = 40
    lam = W.alternating_signs(np.linspace(2.0, 0.1, n))
    A = W.symmetric_spectrum(n, lam, 5)
    out = SP.rsvd_alg5(A, k=10, p=40, seed=2)            # l = n
    ev = np.linalg.eigvalsh(A)
    ref = ev[np.lexsort((-ev, -np.abs(ev)))][:10]
    assert out["l"] == n
    assert np.max(np.abs(out["D"] - ref)) <= 1e-12
    # The selected eigenvectors satisfy A u = lambda u.
    assert np.max(np.abs(A @ out["U"] - out["U"] * out["D"])) <= 1e-11


def _general_exact_rank(m, n, r, seed_u=11, seed_v=12):
    A, sig = W.exact_rank(m, n, r, seed_u, seed_v, top=2.0, ratio=0.75)
    d = min(m, n)
    return A, sig[:r], W.haar(m, d, seed_u)[:, :r], W.haar(n, d, seed_v)[:, :r]


@pytest.mark.parametrize("m,n", [(150, 100), (90, 160)])
def test_alg6_exact_rank_recovers_the_svd(m, n):
    r = 10
    A, sig, U, V = _general_exact_rank(m, n, r)
    out = SP.rsvd_alg6(A, k=r, p=6, seed=4)
    # Eq. (3.14): both equations are consistent, C = Q_c^T A Q_r.
    assert np.max(np.abs(out["C"] - out["Q_c"].T @ A @ out["Q_r"])) <= 1e-11
    assert np.max(np.abs(out["S"] - sig)) <= 1e-12 * sig[0]
    V_fixed = _sign_fix(V)
    sgn = np.sign(np.sum(V_fixed * V, axis=0))
    assert np.max(np.abs(out["Vt"].T - V_fixed)) <= 1e-10
    assert np.max(np.abs(out["U"] - U * sgn[None, :])) <= 1e-10
    assert np.max(np.abs((out["U"] * out["S"]) @ out["Vt"] - A)) <= 1e-11


def test_alg6_full_width_is_an_exact_svd():
    m, n = 70, 50
    sig = W.spectrum_geometric(n, 0.85)
    A = W.known_spectrum(m, n, sig, 3, 4)
    out = SP.rsvd_alg6(A, k=n, p=0, seed=6)              # k = l = min(m, n)
    assert np.max(np.abs(out["S"] - np.linalg.svd(A, compute_uv=False))) <= 1e-12
    assert np.max(np.abs((out["U"] * out["S"]) @ out["Vt"] - A)) <= 1e-12


@pytest.mark.parametrize("alg", [5, 6])
def test_single_pass_respects_eckart_young(alg):
    n = 200
    sig = W.spectrum_geometric(n, 0.9)
    if alg == 5:
        A = W.symmetric_spectrum(n, sig, 13)
        out = SP.rsvd_alg5(A, k=15, p=10, seed=1)
        approx = (out["U"] * out["D"]) @ out["U"].T
    else:
        A = W.known_spectrum(n, n, sig, 13, 14)
        out = SP.rsvd_alg6(A, k=15, p=10, seed=1)
        approx = (out["U"] * out["S"]) @ out["Vt"]
    err = np.linalg.norm(A - approx, 2)
    assert err >= sig[15] * (1 - 1e-12)
    # Single pass is less accurate than the two-pass methods but still near
    # the optimum for a geometric spectrum (statistical, fixed seed).
    assert err <= 20 * sig[15]


# ---- planted mistakes -------------------------------------------------------

def test_pins_pass_unmutated():
    A, sig, _, _ = _general_exact_rank(80, 80, 8)
    out = SP.rsvd_alg6(A, k=8, p=5, seed=2)
    assert np.max(np.abs((out["U"] * out["S"]) @ out["Vt"] - A)) <= 1e-11


def test_transposed_second_sketch_is_caught(monkeypatch):
    """Y_r = A Omega_r (the listing's slip) on a square non-symmetric A."""
    monkeypatch.setattr(SP, "two_sided_sketch", lambda A, Oc, Or: (A @ Oc, A @ Or))
    A, sig, _, _ = _general_exact_rank(80, 80, 8)
    out = SP.rsvd_alg6(A, k=8, p=5, seed=2)
    assert np.max(np.abs((out["U"] * out["S"]) @ out["Vt"] - A)) > 1e-3


def test_sign_error_in_normal_equations_is_caught(monkeypatch):
    def bad(M1, N1, M2, N2):
        import scipy.linalg
        return scipy.linalg.solve_sylvester(M1.T @ M1, M2 @ M2.T, M1.T @ N1 - N2 @ M2.T)
    monkeypatch.setattr(SP, "joint_lstsq", bad)
    rng = np.random.default_rng(2)
    M1, N1 = rng.standard_normal((6, 4)), rng.standard_normal((6, 4))
    M2, N2 = rng.standard_normal((4, 6)), rng.standard_normal((4, 6))
    assert np.max(np.abs(SP.joint_lstsq(M1, N1, M2, N2) - _kron_lstsq(M1, N1, M2, N2))) > 1e-3
