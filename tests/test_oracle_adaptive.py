"""Pins of the adaptive range finder oracle (oracle/adaptive.py) against what
the algorithm guarantees: the returned Q meets the tolerance in the spectral
norm (checked with an exact SVD, for many seeds); the estimate bounds the
true residual from above; an exact-rank-r matrix stops after exactly
ceil(r / b) blocks with a vanishing residual; a smaller tolerance never
gives a smaller basis; and the basis is not much larger than the numerical
rank the tolerance asks for."""

import math

import numpy as np
import pytest

from oracle import adaptive
from paper_2402_17794_amd import workloads as W


def _matrix():
    sig = W.spectrum_geometric(300, 0.9)
    return W.known_spectrum(500, 300, sig, 1, 2), sig


@pytest.mark.parametrize("tol", [1e-1, 1e-3, 1e-6])
def test_meets_tolerance_and_estimate_bounds_residual(tol):
    A, sig = _matrix()
    for seed in range(6):
        out = adaptive.adaptive_range_finder(A, tol, block=8, seed=seed)
        assert out["converged"]
        Q = out["Q"]
        assert np.max(np.abs(Q.T @ Q - np.eye(out["l"]))) <= 1e-12
        res = np.linalg.svd(A - Q @ (Q.T @ A), compute_uv=False)[0]
        assert res <= tol
        assert res <= out["est"]
        # the basis is not much larger than needed: sigma_{l - 2b} is above tol / 100
        if out["l"] > 16:
            assert sig[out["l"] - 17] > tol / 100


@pytest.mark.parametrize("r,b", [(12, 8), (16, 16), (5, 16), (30, 16)])
def test_exact_rank_is_found_exactly(r, b):
    """rank r with sigma_r = 0.7^(r-1) >= 2e-5: every block appends only its
    independent directions, so l = r after ceil(r / b) blocks and the next
    block stops with a vanishing residual."""
    A, _ = W.exact_rank(400, 250, r, 3, 4)
    out = adaptive.adaptive_range_finder(A, 1e-10, block=b, seed=1)
    assert out["converged"] and out["l"] == r
    assert out["blocks"] == math.ceil(r / b) + 1
    Q = out["Q"]
    assert np.max(np.abs(Q.T @ Q - np.eye(r))) <= 1e-12
    assert np.linalg.norm(A - Q @ (Q.T @ A)) <= 1e-12 * np.linalg.norm(A)


def test_smaller_tolerance_never_gives_a_smaller_basis():
    A, _ = _matrix()
    ls = [adaptive.adaptive_range_finder(A, tol, block=8, seed=2)["l"] for tol in (1e-1, 1e-2, 1e-4, 1e-8)]
    assert ls == sorted(ls)


def test_cap_reports_not_converged():
    A, _ = _matrix()
    out = adaptive.adaptive_range_finder(A, 1e-14, block=16, max_l=64, seed=0)
    assert not out["converged"] and 48 < out["l"] <= 64 and out["est"] > 1e-14
