"""Pins for the oracle's Algorithm 4 end to end.

Nothing here compares the oracle with itself.  The pins are what the paper
and the mathematics fix:
* l = min(m, n): the randomized SVD becomes an exact SVD, so the singular
  values are the generator's and the vectors LAPACK's (library special case);
* exact rank r <= l: the range is captured exactly (zero residual, exact
  singular values);
* interlacing: sigma_i(Q^T A) <= sigma_i(A); Eckart-Young, eq. (3.1):
  ||A - QQ^T A||_2 >= sigma_{l+1} for every seed;
* the expected-error bounds of Theorems 2, 3, 6 and eq. (3.5), averaged over
  many seeds on the eq. (4.1) test family (Section 4.2 grids);
* eq. (3.2): after q power steps range(Q) = range(U Sigma^(2q+1) V^T Omega),
  built from the generator's own factors; Algorithm 3 and Algorithm 4 give
  the same range in exact arithmetic (they differ only in round-off);
* the outputs' defining identities: orthonormal U, V, Q B = U Sigma V^T for
  the full rank-l factorisation, descending sigma, the sign convention.
"""

import numpy as np
import pytest

from oracle import bounds
from oracle.philox import omega
from oracle.rsvd import residual_norms, rsvd_alg3, rsvd_alg4
from paper_2402_17794_amd import workloads as W


def _orth_err(Q):
    return np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1])))


def _sin_theta(Q1, Q2):
    """Largest sine of the canonical angles between range(Q1), range(Q2)."""
    return float(np.linalg.norm(Q2 - Q1 @ (Q1.T @ Q2), 2))


@pytest.mark.parametrize("m,n,q", [(60, 40, 0), (40, 60, 1), (50, 50, 2)])
def test_full_width_is_exact_svd(m, n, q):
    d = min(m, n)
    sig = W.spectrum_geometric(d, 0.8)
    A = W.known_spectrum(m, n, sig, 11, 12)
    out = rsvd_alg4(A, k=d, p=5, q=q, seed=3)
    assert out["l"] == d
    assert np.max(np.abs(out["S"] - sig)) <= 1e-12 * sig[0]
    Ul, sl, Vtl = np.linalg.svd(A, full_matrices=False)
    top = 10                                      # well-separated leading pairs
    for i in range(top):
        su = np.sign(out["U"][:, i] @ Ul[:, i])
        assert np.max(np.abs(out["U"][:, i] - su * Ul[:, i])) <= 1e-9
        assert np.max(np.abs(out["Vt"][i] - su * Vtl[i])) <= 1e-9


@pytest.mark.parametrize("r,k,p,q", [(8, 8, 5, 0), (8, 5, 10, 1), (20, 20, 0, 0)])
def test_exact_rank_recovery(r, k, p, q):
    A, sig = W.exact_rank(300, 120, r, 5, 6)
    out = rsvd_alg4(A, k=k, p=p, q=q, seed=9)
    spec, fro = residual_norms(A, out["Q"])
    assert spec <= 1e-12 * sig[0] and fro <= 1e-12 * sig[0]
    assert np.max(np.abs(out["S"] - sig[:k])) <= 1e-12 * sig[0]


@pytest.mark.parametrize("seed", range(6))
def test_interlacing_and_eckart_young(seed):
    sig = W.eq41_spectrum(300, 10.0)
    A = W.known_spectrum(3000, 300, sig, 1, 2)
    k, p, q = 20, 5, seed % 2
    out = rsvd_alg4(A, k, p, q, seed=seed, return_full_l=True)
    l = out["l"]
    assert np.all(out["S"] <= sig[:l] * (1 + 1e-12))
    spec, _ = residual_norms(A, out["Q"])
    assert spec >= bounds.eckart_young_floor(sig, l) * (1 - 1e-10)


def _mean_residual(A, k, p, q, seeds):
    vals = []
    for s in seeds:
        out = rsvd_alg4(A, k, p, q, seed=s)
        vals.append(residual_norms(A, out["Q"])[0])
    return float(np.mean(vals)), vals


@pytest.fixture(scope="module")
def eq41_gap10():
    sig = W.eq41_spectrum(300, 10.0)
    return W.known_spectrum(3000, 300, sig, 1, 2), sig


@pytest.mark.parametrize("k,p", [(5, 5), (20, 5), (30, 5), (20, 15), (20, 25)])
def test_expected_error_bounds_q0(eq41_gap10, k, p):
    """Theorem 2 (Algorithm 1 / 2 at q = 0) and Theorem 6 at q = 0, on the
    Section 4.2 grid (gap = 10), mean over 30 seeds."""
    A, sig = eq41_gap10
    mean, vals = _mean_residual(A, k, p, 0, range(30))
    assert mean <= bounds.thm2(sig, k, p, 3000, 300)
    assert mean <= bounds.thm6(sig, k, p, 0)
    assert min(vals) >= bounds.eckart_young_floor(sig, k + p) * (1 - 1e-10)


@pytest.mark.parametrize("k,p,q", [(5, 5, 1), (20, 5, 1), (20, 15, 1), (10, 5, 2)])
def test_expected_error_bounds_power(eq41_gap10, k, p, q):
    """Theorems 3 and 6 for the power scheme, mean over 30 seeds."""
    A, sig = eq41_gap10
    mean, _ = _mean_residual(A, k, p, q, range(30))
    assert mean <= bounds.thm3(sig, k, p, q, 3000, 300)
    assert mean <= bounds.thm6(sig, k, p, q)


def test_expected_error_bound_100_runs_flat_tail():
    """100 runs at k = 20, p = 5 (as in Section 4.2), on a spectrum that is
    flat after k so eq. (3.5) applies, for q = 0 and q = 1."""
    m, n, k, p = 600, 120, 20, 5
    sig = np.concatenate([np.linspace(1.0, 0.5, k), np.full(n - k, 0.1)])
    A = W.known_spectrum(m, n, sig, 3, 4)
    for q in (0, 1):
        mean, vals = _mean_residual(A, k, p, q, range(100))
        assert mean <= bounds.eq35(sig[k], k, p, q, m, n)
        assert mean <= bounds.thm6(sig, k, p, q) * (1 + 1e-12)
        assert min(vals) >= sig[k + p] * (1 - 1e-10)


@pytest.mark.parametrize("q", [1, 2])
def test_power_scheme_range_matches_eq32(q):
    """Eq. (3.2): A^(q) = (A A^T)^q A = U Sigma^(2q+1) V^T.  Built from the
    generator's own U, Sigma, V (not from A), its range applied to Omega
    must be the range Algorithm 4 finds."""
    m, n, l = 200, 80, 12
    d = min(m, n)
    sig = W.spectrum_geometric(d, 0.9)
    U = W.haar(m, d, 21)
    V = W.haar(n, d, 22)
    A = (U * sig) @ V.T
    out = rsvd_alg4(A, k=l, p=0, q=q, seed=4)
    Yq = (U * sig ** (2 * q + 1)) @ (V.T @ omega(4, n, l))
    Qref, _ = np.linalg.qr(Yq)
    assert _sin_theta(out["Q"], Qref) <= 1e-8


def test_algorithm3_and_algorithm4_same_range():
    sig = W.spectrum_geometric(100, 0.9)
    A = W.known_spectrum(300, 100, sig, 7, 8)
    a3 = rsvd_alg3(A, 10, 5, 1, seed=2)
    a4 = rsvd_alg4(A, 10, 5, 1, seed=2)
    assert _sin_theta(a3["Q"], a4["Q"]) <= 1e-10
    assert np.max(np.abs(a3["S"] - a4["S"])) <= 1e-12


def test_output_identities_and_signs():
    A = W.eq41_matrix(2.0, 5, 6)
    out = rsvd_alg4(A, k=25, p=5, q=1, seed=1, return_full_l=True)
    U, S, Vt, Q, B = out["U"], out["S"], out["Vt"], out["Q"], out["B"]
    assert _orth_err(U) <= 1e-12 and _orth_err(Vt.T) <= 1e-12 and _orth_err(Q) <= 1e-12
    assert np.all(np.diff(S) <= 0)
    assert np.linalg.norm(Q @ B - (U * S) @ Vt) <= 1e-12 * np.linalg.norm(B)
    assert np.max(np.abs(B - Q.T @ A)) == 0.0
    for i in range(Vt.shape[0]):
        idx = int(np.argmax(np.abs(Vt[i])))
        assert Vt[i, idx] > 0
    short = rsvd_alg4(A, k=25, p=5, q=1, seed=1)
    assert short["U"].shape == (3000, 25) and short["Vt"].shape == (25, 300)
    assert np.array_equal(short["S"], S[:25])


def test_validation_and_edge_cases():
    A = np.random.default_rng(0).standard_normal((30, 20))
    for bad in [dict(k=0, p=1, q=0), dict(k=21, p=0, q=0), dict(k=2, p=-1, q=0), dict(k=2, p=1, q=-1)]:
        with pytest.raises(ValueError):
            rsvd_alg4(A, **bad)
    out = rsvd_alg4(A, k=15, p=10, q=1)            # k + p > min(m, n): l clamps
    assert out["l"] == 20
    out0 = rsvd_alg4(A, k=5, p=0, q=0)             # p = 0 allowed
    assert out0["l"] == 5 and out0["U"].shape == (30, 5)
    z = rsvd_alg4(np.zeros((25, 10)), k=3, p=2, q=1)
    assert np.all(z["S"] == 0.0)
    assert _orth_err(z["Q"]) == 0.0


def test_seed_determinism_and_omega_override():
    A = W.eq41_matrix(1.0, 1, 2)
    a = rsvd_alg4(A, 10, 5, 1, seed=42)
    b = rsvd_alg4(A, 10, 5, 1, seed=42)
    c = rsvd_alg4(A, 10, 5, 1, omega=omega(42, 300, 15))
    assert np.array_equal(a["U"], b["U"]) and np.array_equal(a["U"], c["U"])
    d = rsvd_alg4(A, 10, 5, 1, seed=43)
    assert not np.allclose(a["U"], d["U"]) or not np.allclose(a["S"], d["S"], rtol=0, atol=0)


# ---- spectral-norm estimator (block power iteration with Rayleigh-Ritz) ----
# Pins: when rank(E) <= block, one iteration puts range(E^T) inside range(Z),
# so the Ritz value is sigma_1(E) exactly (library SVD); with a gap the
# estimate converges to sigma_1; it never exceeds sigma_1 (a Ritz value of
# E^T E on an orthonormal block), for any number of iterations.

@pytest.mark.parametrize("m,n,rank", [(200, 60, 10), (60, 200, 16), (150, 150, 1)])
def test_spectral_estimator_exact_when_rank_within_block(m, n, rank):
    from oracle.rsvd import spectral_norm_power
    A, _ = W.exact_rank(m, n, rank, 3, 4, top=2.0, ratio=0.8)
    exact = np.linalg.svd(A, compute_uv=False)[0]
    assert abs(spectral_norm_power(A, iters=1, block=16, seed=5) - exact) <= 1e-12 * exact


def test_spectral_estimator_converges_and_bounds():
    from oracle.rsvd import spectral_norm_power
    sig = np.concatenate([[1.0], 0.5 * W.spectrum_geometric(79, 0.97)])     # gap after sigma_1
    A = W.known_spectrum(300, 80, sig, 7, 8)
    assert abs(spectral_norm_power(A, iters=30, block=16, seed=1) - 1.0) <= 1e-12
    rng = np.random.default_rng(4)
    for t in range(4):
        G = rng.standard_normal((120, 90))
        s1 = np.linalg.svd(G, compute_uv=False)[0]
        for iters in (0, 1, 3):
            est = spectral_norm_power(G, iters=iters, block=16, seed=t)
            assert est <= s1 * (1 + 1e-13)
            assert est >= 0.5 * s1


def test_alg4_beats_alg3_at_large_q():
    """Section 3.3: without orthonormalisation between the products of the
    power scheme, round-off erases the information of the smaller singular
    values as q grows, which Algorithm 4 avoids.  Eq. (4.1) stand-in with a
    gap of 10 after sigma_15, k = 20, p = 5, FP64: the two agree at q = 1;
    Algorithm 4's error keeps decreasing with q, while Algorithm 3's grows
    from q = 3 on and is several times larger at q = 8."""
    A = W.eq41_matrix(10.0, 1, 2)
    e3 = {q: residual_norms(A, rsvd_alg3(A, 20, 5, q, seed=0)["Q"])[0] for q in (1, 2, 4, 8)}
    e4 = {q: residual_norms(A, rsvd_alg4(A, 20, 5, q, seed=0)["Q"])[0] for q in (1, 2, 4, 8)}
    assert abs(e3[1] - e4[1]) <= 1e-8 * e4[1]
    assert e4[8] <= e4[4] <= e4[2] <= e4[1]
    assert e3[4] > e3[2] and e3[8] > 3.0 * e4[8]
