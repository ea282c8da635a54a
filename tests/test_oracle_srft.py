"""Pins of the SRFT oracle (oracle/srft.py) against what the definition and
independent libraries fix: the orthogonality Omega^T Omega = (n/l) I (exact,
from the orthogonality of D and F and distinct sampled columns), the DCT-II
columns against scipy's orthonormal DCT of the identity, distinctness and
uniformity of Floyd's sample, the sign statistics, and exact range recovery
for exact-rank inputs (FastRandRF)."""

import numpy as np
import pytest
from scipy import fft as sfft
from scipy import stats

from oracle import srft
from oracle.linalg import householder_qr
from paper_2402_17794_amd import workloads as W


@pytest.mark.parametrize("n,l,seed", [(64, 10, 0), (1000, 110, 3), (257, 257, 1), (4096, 272, 9)])
def test_columns_orthogonal_with_norm_n_over_l(n, l, seed):
    Om = srft.srft_omega(seed, n, l)
    assert np.max(np.abs(Om.T @ Om - (n / l) * np.eye(l))) <= 1e-12 * (n / l)


@pytest.mark.parametrize("n", [1, 7, 64, 1000])
def test_dct_columns_equal_scipy_orthonormal_dct(n):
    F = sfft.dct(np.eye(n), type=2, norm="ortho", axis=0).T      # rows: sample index i, columns: frequency c
    for c in range(n):
        assert np.max(np.abs(srft.dct2_column(n, c) - F[:, c])) <= 1e-13


def test_omega_is_scaled_signed_dct_columns_via_fast_transform():
    """A Omega through a fast transform: (A D) F, computed with scipy's DCT of
    the rows of A D, then the sampled columns, times sqrt(n/l)."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((30, 500))
    n, l = 500, 40
    d = srft.srft_signs(5, n)
    cols = srft.srft_columns(5, n, l)
    fast = np.sqrt(n / l) * sfft.dct(A * d[None, :], type=2, norm="ortho", axis=1)[:, cols]
    assert np.max(np.abs(A @ srft.srft_omega(5, n, l) - fast)) <= 1e-12 * np.abs(fast).max()


@pytest.mark.parametrize("n,l", [(10, 10), (100, 3), (8192, 110), (5, 1)])
def test_floyd_sample_distinct_in_range(n, l):
    cols = srft.srft_columns(2, n, l)
    assert cols.shape == (l,) and len(set(cols.tolist())) == l
    assert cols.min() >= 0 and cols.max() < n


def test_floyd_sample_uniform():
    """Each of 20 columns is taken with probability l/n = 0.25: counts over
    2000 seeds against the binomial."""
    n, l, seeds = 20, 5, 2000
    counts = np.zeros(n)
    for s in range(seeds):
        counts[srft.srft_columns(s, n, l)] += 1
    expected = seeds * l / n
    chi2 = np.sum((counts - expected) ** 2 / expected)
    assert stats.chi2.sf(chi2, n - 1) > 1e-4


def test_signs_balanced_and_independent_of_columns():
    d = srft.srft_signs(11, 100000)
    assert set(np.unique(d).tolist()) == {-1.0, 1.0}
    assert abs(d.mean()) < 5.0 / np.sqrt(d.size)
    assert not np.array_equal(srft.srft_signs(11, 64), srft.srft_signs(12, 64))


def test_fast_range_finder_recovers_exact_rank():
    A, sig = W.exact_rank(600, 300, 12, 3, 4)
    Q, _ = srft.fast_range_finder(A, 40, seed=2)
    assert np.max(np.abs(Q.T @ Q - np.eye(40))) <= 1e-12
    assert np.linalg.norm(A - Q @ (Q.T @ A)) <= 1e-12 * np.linalg.norm(A)


def test_a_wrong_dct_scale_or_index_fails_the_pins():
    """Mutations: DCT columns without the sqrt(2/n) normalisation break the
    orthogonality pin; the frequency index off by one (still an orthonormal
    basis) breaks the comparison with scipy's DCT."""
    n, l = 200, 20
    d = srft.srft_signs(1, n)
    cols = srft.srft_columns(1, n, l)
    i = np.arange(n)
    bad1 = np.stack([d * np.cos(np.pi * (2 * i + 1) * c / (2 * n)) for c in cols], axis=1) * np.sqrt(n / l)
    assert np.max(np.abs(bad1.T @ bad1 - (n / l) * np.eye(l))) > 1e-6
    F = sfft.dct(np.eye(n), type=2, norm="ortho", axis=0).T
    shifted = lambda c: np.sqrt(2.0 / n) * np.cos(np.pi * (2.0 * i + 1.0) * (c + 1) / (2.0 * n))
    assert max(np.max(np.abs(shifted(c) - F[:, c])) for c in range(1, n - 1)) > 1e-3
