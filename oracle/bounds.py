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


def thm5(sigma, k, q, Omega, V):
    """Theorem 5 (under Assumption 4): bounds on the sines of the canonical
    angles theta_j between range(U_k) and the left space of the power-scheme
    sketch, and v_j between range(V_k) and the right space, j = 1..k:

      sin theta_j <= g_j^(2q+1) c / sqrt(1 + g_j^(4q+2) c^2),
      sin v_j     <= g_j^(2q+2) c / sqrt(1 + g_j^(4q+4) c^2),

    with g_j = sigma_{k+1} / sigma_j (gamma_j, the reading of gamma for index
    j) and c = ||Omega_2 Omega_1^+||_2, where V^T Omega = [Omega_1; Omega_2]
    splits the test matrix along the first k right singular vectors (V: all
    right singular vectors of A, n x min(m, n) or n x n).  Returns (bounds
    for theta, bounds for v), each of length k."""
    sigma = np.asarray(sigma, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    Om = np.asarray(Omega, dtype=np.float64)
    O1 = V[:, :k].T @ Om
    O2 = V[:, k:].T @ Om
    c = float(np.linalg.norm(O2 @ np.linalg.pinv(O1), 2))
    g = np.array([_s(sigma, k + 1) / _s(sigma, j) for j in range(1, k + 1)])
    e1, e2 = 2 * q + 1, 2 * q + 2
    bt = g ** e1 * c / np.sqrt(1.0 + g ** (2 * e1) * c * c)
    bv = g ** e2 * c / np.sqrt(1.0 + g ** (2 * e2) * c * c)
    return bt, bv
