"""Expected-error bounds and the optimal-error floor (test infrastructure only).

All functions take the singular values of A as a 1-based sequence stored in a
0-based array: sigma[0] is sigma_1.  They return the bound on
E||A - Q Q^T A||_2 that the cited theorem states.
"""

import math

import numpy as np


def _s(sigma, i):
    """sigma_i (1-based); zero past the end of the spectrum."""
    sigma = np.asarray(sigma, dtype=np.float64)
    return float(sigma[i - 1]) if i - 1 < sigma.size else 0.0


def eckart_young_floor(sigma, l):
    """Eq. (3.1): no rank-l approximation beats sigma_{l+1}, so
    ||A - Q Q^T A||_2 >= sigma_{l+1} for every m x l orthonormal Q."""
    return _s(sigma, l + 1)


def thm2(sigma, k, p, m, n):
    """Theorem 2 (Algorithm 1, q = 0): [1 + 4 sqrt(k+p)/(p-1) sqrt(min(m,n))]
    sigma_{k+1}.  Needs k >= 2, p >= 2, k + p <= min(m, n)."""
    return (1.0 + 4.0 * math.sqrt(k + p) / (p - 1) * math.sqrt(min(m, n))) * _s(sigma, k + 1)


def thm3(sigma, k, p, q, m, n):
    """Theorem 3 (power scheme): [1 + 4 sqrt((k+p) min(m,n))/(p-1)]^(1/(2q+1))
    sigma_{k+1}."""
    c = 1.0 + 4.0 * math.sqrt((k + p) * min(m, n)) / (p - 1)
    return c ** (1.0 / (2 * q + 1)) * _s(sigma, k + 1)


def thm6(sigma, k, p, q):
    """Theorem 6, eq. (3.4): [(1 + sqrt(k/(p-1))) sigma_{k+1}^(2q+1)
    + e sqrt(k+p)/p (sum_{j>k} sigma_j^(2(2q+1)))^(1/2)]^(1/(2q+1))."""
    sigma = np.asarray(sigma, dtype=np.float64)
    e = 2 * q + 1
    tail = sigma[k:]
    head = (1.0 + math.sqrt(k / (p - 1))) * _s(sigma, k + 1) ** e
    rest = math.e * math.sqrt(k + p) / p * math.sqrt(float(np.sum(tail ** (2 * e))))
    return (head + rest) ** (1.0 / e)


def eq35(sigma_k1, k, p, q, m, n):
    """Eq. (3.5), the flat-tail case of eq. (3.4): [(1 + sqrt(k/(p-1)))
    + e sqrt(k+p)/p sqrt(min(m,n) - k)]^(1/(2q+1)) sigma_{k+1}."""
    c = (1.0 + math.sqrt(k / (p - 1))) + math.e * math.sqrt(k + p) / p * math.sqrt(min(m, n) - k)
    return c ** (1.0 / (2 * q + 1)) * sigma_k1
