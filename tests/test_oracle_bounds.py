"""Pins for the bound formulas: relations the paper states between them."""

import math

import numpy as np
import pytest

from oracle import bounds


@pytest.mark.parametrize("k,p,m,n", [(5, 5, 3000, 300), (20, 10, 512, 256), (100, 10, 8192, 8192)])
def test_thm3_at_q0_equals_thm2(k, p, m, n):
    sig = 1.0 / np.arange(1, min(m, n) + 1)
    assert bounds.thm3(sig, k, p, 0, m, n) == pytest.approx(bounds.thm2(sig, k, p, m, n), rel=1e-14)


@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_eq34_with_flat_tail_is_eq35(q):
    k, p, m, n = 20, 5, 3000, 300
    sig = np.concatenate([np.linspace(3.0, 1.0, k), np.full(n - k, 0.25)])
    assert bounds.thm6(sig, k, p, q) == pytest.approx(bounds.eq35(0.25, k, p, q, m, n), rel=1e-13)


def test_power_drives_factor_to_one():
    """Section 3.2: the factor in front of sigma_{k+1} tends to 1 as q grows."""
    k, p, m, n = 20, 5, 3000, 300
    f = [bounds.thm3([1.0] * 300, k, p, q, m, n) for q in range(0, 30)]
    assert all(a > b for a, b in zip(f, f[1:]))
    assert f[-1] < 1.2 and f[0] > 10


def test_floor_and_hand_values():
    sig = 0.8 ** np.arange(1, 257)
    assert bounds.eckart_young_floor(sig, 30) == sig[30]
    assert bounds.eckart_young_floor(sig, 256) == 0.0
    # Theorem 2 for k = 20, p = 10, 512 x 256, sigma_21 = 0.8^21
    expect = (1 + 4 * math.sqrt(30) / 9 * math.sqrt(256)) * 0.8 ** 21
    assert bounds.thm2(sig, 20, 10, 512, 256) == pytest.approx(expect, rel=1e-14)
