"""Subsampled randomized trigonometric test matrix (SRFT) and the fast range
finder built on it.  Test infrastructure only (see the package docstring).

The thesis (Appendix A, FastRandRF and its sub-function SRFT) draws the
n x l test matrix as Omega = sqrt(n / l) D F R with D an n x n diagonal of
independent entries uniform on the complex unit circle, F the n x n unitary
discrete Fourier transform and R an n x l matrix that samples l coordinates
uniformly at random; FastRandRF forms Y = A Omega and an orthonormal basis of
its range.  Reading for real data (the path is real throughout): D has
independent +-1 entries (the real unit circle), F is the orthonormal DCT-II,
the real orthogonal counterpart of the unitary DFT,

  F[i, c] = sqrt(1 / n)                               (c = 0)
          = sqrt(2 / n) cos(pi (2 i + 1) c / (2 n))   (c >= 1),

and R picks l distinct columns of F.  Omega then has orthogonal columns with
Omega^T Omega = (n / l) I exactly.

Random numbers (Philox4x32-10 as in oracle.philox, stream 4, key = seed):
  * d_i = -1 if bit 0 of word (i mod 4) of block (i // 4, 0, 4, 0) is set,
    else +1;
  * the column sample by Floyd's algorithm: for t = 0 .. l-1, with
    j = n - l + t, draw x = floor(w (j + 1) / 2^32) from word 0 w of block
    (t, 1, 4, 0), a uniform integer in [0, j]; take x if it was not taken
    before, else j.  The sampled columns r_0 .. r_{l-1} are in this order.
"""

import numpy as np

from .linalg import orth
from .philox import philox4

SRFT_STREAM = 4


def _key(seed):
    seed = int(seed)
    return np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)


def srft_signs(seed, n):
    """The diagonal of D: n values +-1."""
    g = np.arange((n + 3) // 4, dtype=np.uint64)
    ctr = np.stack([g, 0 * g, 0 * g + SRFT_STREAM, 0 * g], axis=-1)
    w = philox4(ctr, _key(seed)).reshape(-1)[:n]
    return np.where(w & np.uint64(1), -1.0, 1.0)


def srft_columns(seed, n, l):
    """The l sampled columns of F (distinct, in [0, n)), by Floyd's algorithm."""
    if not 0 <= l <= n:
        raise ValueError("need 0 <= l <= n")
    t = np.arange(l, dtype=np.uint64)
    ctr = np.stack([t, 0 * t + 1, 0 * t + SRFT_STREAM, 0 * t], axis=-1)
    w = philox4(ctr, _key(seed))[:, 0] if l else np.zeros(0, np.uint64)
    chosen, cols = set(), []
    for step in range(l):
        j = n - l + step
        x = int((int(w[step]) * (j + 1)) >> 32)
        pick = x if x not in chosen else j
        chosen.add(pick)
        cols.append(pick)
    return np.array(cols, dtype=np.int64)


def dct2_column(n, c):
    """Column c of the orthonormal DCT-II matrix F (length n).  The cosine's
    argument pi (2 i + 1) c / (2 n) is reduced modulo 2 pi in exact integer
    arithmetic first (the same function, evaluated without the rounding of
    a large argument)."""
    if c == 0:
        return np.full(n, np.sqrt(1.0 / n))
    i = np.arange(n, dtype=np.int64)
    m = ((2 * i + 1) * int(c)) % (4 * n)
    return np.sqrt(2.0 / n) * np.cos(np.pi * m.astype(np.float64) / (2.0 * n))


def srft_omega(seed, n, l):
    """Omega = sqrt(n / l) D F R, n x l."""
    d = srft_signs(seed, n)
    cols = srft_columns(seed, n, l)
    out = np.empty((n, l), dtype=np.float64)
    for t, c in enumerate(cols):
        out[:, t] = np.sqrt(n / l) * d * dct2_column(n, int(c))
    return out


def fast_range_finder(A, l, seed=0):
    """FastRandRF: Y = A Omega with the SRFT test matrix, Q = orth(Y)."""
    A = np.asarray(A, dtype=np.float64)
    Om = srft_omega(seed, A.shape[1], l)
    return orth(A @ Om), Om


__all__ = ["srft_signs", "srft_columns", "dct2_column", "srft_omega", "fast_range_finder", "SRFT_STREAM"]
