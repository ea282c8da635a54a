"""Philox4xW-R counter-based generator and the Gaussian test matrix.

Test infrastructure only (see the package docstring).

The paper draws the n x (k+p) test matrix Omega with i.i.d. standard normal
entries (Algorithm 4 step 1; "standard Gaussian" in Theorems 2 and 3) and
leaves the generator to the host language.  The reading used here (so that a
solve is a pure function of its seed) is:

* uniform bits from Philox4x32-10, as published by Salmon, Moraes, Dror and
  Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 4-word
  counter block and a 2-word key; each round multiplies words 0 and 2 by two
  fixed odd constants, takes the high and low halves of the double-width
  products, xors the high halves with the other two words and the key, and
  permutes; between rounds the key is bumped by two Weyl constants (the
  fractional parts of the golden ratio and of sqrt(3), in W-bit fixed point);
* normals by the Box-Muller transform of pairs of 24-bit uniforms.

The generator is written once for any word width W (32 or 64) so that the
64-bit instance can be checked against an independent library implementation
of Philox4x64-10; the 32-bit instance is the one Omega uses.
"""

import numpy as np

# Multipliers and Weyl key increments of Philox4xW (SC'11, Table of constants).
_CONSTANTS = {
    32: dict(M0=0xD2511F53, M1=0xCD9E8D57,
             W0=0x9E3779B9, W1=0xBB67AE85),
    64: dict(M0=0xD2E7470EE14C6C93, M1=0xCA5A826395121157,
             W0=0x9E3779B97F4A7C15, W1=0xBB67AE8584CAA73B),
}

_U64 = np.uint64


def _mask(width):
    return _U64((1 << width) - 1) if width < 64 else _U64(0xFFFFFFFFFFFFFFFF)


def mulhilo(a, b, width):
    """High and low W-bit halves of the 2W-bit product a*b (schoolbook on
    W/2-bit limbs, so every partial product fits in 64 bits)."""
    a = np.asarray(a, dtype=_U64)
    b = np.asarray(b, dtype=_U64)
    h = _U64(width // 2)
    lm = _U64((1 << (width // 2)) - 1)
    a0, a1 = a & lm, a >> h
    b0, b1 = b & lm, b >> h
    with np.errstate(over="ignore"):
        p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
        mid = (p00 >> h) + (p01 & lm) + (p10 & lm)
        lo = (p00 & lm) | ((mid & lm) << h)
        hi = p11 + (p01 >> h) + (p10 >> h) + (mid >> h)
    m = _mask(width)
    return hi & m, lo & m


def philox4(counter, key, width=32, rounds=10):
    """Philox4xW-R block function.

    counter: array (..., 4) of W-bit words; key: array (..., 2) of W-bit words
    (broadcastable).  Returns an array (..., 4) of W-bit words.
    """
    c = _CONSTANTS[width]
    m = _mask(width)
    ctr = np.asarray(counter, dtype=_U64)
    k = np.asarray(key, dtype=_U64)
    x0, x1, x2, x3 = (ctr[..., i] & m for i in range(4))
    k0, k1 = k[..., 0] & m, k[..., 1] & m
    M0, M1 = _U64(c["M0"]), _U64(c["M1"])
    W0, W1 = _U64(c["W0"]), _U64(c["W1"])
    with np.errstate(over="ignore"):        # arithmetic is modulo 2^64 by design
        for r in range(rounds):
            if r > 0:
                k0 = (k0 + W0) & m
                k1 = (k1 + W1) & m
            hi0, lo0 = mulhilo(M0, x0, width)
            hi1, lo1 = mulhilo(M1, x2, width)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack(np.broadcast_arrays(x0, x1, x2, x3), axis=-1)


def uniform_pair(a, b):
    """Two uniforms from two 32-bit words, both exact in float32 and float64:
    u1 = (top 24 bits of a + 1) / 2^24 in (0, 1]  (safe for the logarithm),
    u2 = (top 24 bits of b) / 2^24     in [0, 1)."""
    a = np.asarray(a, dtype=_U64)
    b = np.asarray(b, dtype=_U64)
    u1 = ((a >> _U64(8)) + _U64(1)).astype(np.float64) * 2.0 ** -24
    u2 = (b >> _U64(8)).astype(np.float64) * 2.0 ** -24
    return u1, u2


def box_muller(u1, u2):
    """Box-Muller: (r cos 2 pi u2, r sin 2 pi u2) with r = sqrt(-2 ln u1)."""
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)


def omega(seed, n, l, stream=0):
    """The n x l Gaussian test matrix of Algorithm 4 step 1.

    Element (i, j) comes from the Philox4x32-10 block with
    counter = (i // 4, j, stream, 0) and key = (low 32 bits of seed,
    high 32 bits of seed).  Rows 4g, 4g+1 use the Box-Muller pair built from
    words (0, 1) of block (g, j); rows 4g+2, 4g+3 the pair from words (2, 3).
    The even row of a pair takes the cosine branch, the odd row the sine.
    Column j does not depend on l, so a narrower Omega is a prefix of a wider
    one.
    """
    seed = int(seed)
    n, l = int(n), int(l)
    out = np.zeros((n, l), dtype=np.float64)
    if n == 0 or l == 0:
        return out
    groups = (n + 3) // 4
    g = np.arange(groups, dtype=_U64)[:, None]
    j = np.arange(l, dtype=_U64)[None, :]
    ctr = np.stack(np.broadcast_arrays(g, j, _U64(stream) + 0 * g, 0 * g + 0 * j), axis=-1)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=_U64)
    x = philox4(ctr, key, width=32, rounds=10)          # (groups, l, 4)
    u1a, u2a = uniform_pair(x[..., 0], x[..., 1])
    u1b, u2b = uniform_pair(x[..., 2], x[..., 3])
    z0, z1 = box_muller(u1a, u2a)
    z2, z3 = box_muller(u1b, u2b)
    full = np.stack([z0, z1, z2, z3], axis=1).reshape(groups * 4, l)
    out[:] = full[:n]
    return out


def philox_words(seed, ctr_rows, stream=0):
    """Raw uint32 words for counter blocks (g, j, stream, 0) given as an array
    of (g, j) pairs; used to compare the bit streams of two implementations."""
    ctr_rows = np.asarray(ctr_rows, dtype=_U64)
    g, j = ctr_rows[:, 0], ctr_rows[:, 1]
    ctr = np.stack([g, j, np.full_like(g, stream), np.zeros_like(g)], axis=-1)
    key = np.array([int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF], dtype=_U64)
    return philox4(ctr, key, width=32, rounds=10).astype(np.uint32)
