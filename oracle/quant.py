"""Oracle for the low-precision storage of A (test infrastructure; see the
package header).  Plain numpy, following the definitions stated below.

The thesis computes in double precision throughout and fixes no storage
format; these definitions are the reading this project takes for the BF16
and FP8 forms of the randomized SVD:

* BF16: round to nearest, ties to even, of the FP32 value to 8 significant
  bits (the upper 16 bits of the FP32 pattern); NaN -> 0x7FC0.
* FP8 E4M3 (OCP "E4M3FN": exponent bias 7, 3 mantissa bits, no infinity,
  0x7F / 0xFF NaN, largest finite 448): round to nearest, ties to even;
  |x| >= 448 saturates to +-448; |x| < 2^-6 is a multiple of 2^-9.
* Column-scaled FP8 matrix: amax_j = max_i |A_ij|; s_j = amax_j / 448 and
  inv_j = 448 / amax_j, each rounded in FP32 (1 and 1 for a zero column);
  Aq_ij = e4m3(fl32(A_ij * inv_j)); the represented matrix is Aq diag(s).
* The skinny operand X of a product with such a matrix (GPU internals,
  replicated here so a product can be checked bit for bit up to the
  summation order):
    A X   (FP8): X'_jc = fl32(s_j X_jc), then each column is scaled like a
          matrix column: t_c = amax_c(X') / 448, Xq = e4m3(X' * 448/amax_c);
          the product is t_c * (Aq Xq)_ic.
    A^T Y (FP8): Yq = column-scaled e4m3 of Y with t_c; product s_j t_c (Aq^T Yq)_jc.
    BF16: X -> bf16(X), no scales.
"""

import numpy as np

E4M3_MAX = 448.0


def bf16_bits(x):
    """uint16 BF16 patterns of float32 x (round to nearest even)."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    return np.where(nan, 0x7FC0, r).astype(np.uint16)


def bf16_value(bits):
    """float32 values of uint16 BF16 patterns."""
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def e4m3_bits(x):
    """uint8 E4M3 patterns of float32 x (round to nearest even, saturating)."""
    x = np.asarray(x, dtype=np.float32)
    u = np.ascontiguousarray(x).view(np.uint32)
    sign = ((u >> 24) & 0x80).astype(np.uint8)
    a = np.abs(x)
    e = ((u >> 23) & 0xFF).astype(np.int64) - 127
    with np.errstate(over="ignore", invalid="ignore"):
        q_sub = np.rint(a * np.float32(512.0))
        q_norm = np.rint(np.ldexp(a, (3 - np.clip(e, -6, 200)).astype(np.int32)))
    # lanes of the other branch (or non-finite inputs) may hold inf / NaN: zero them before casting
    q_sub = np.where(np.isfinite(q_sub), q_sub, 0.0)
    q_norm = np.where(np.isfinite(q_norm), q_norm, 8.0)
    up = q_norm == 16
    e_n = np.where(up, e + 1, e)
    q_n = np.where(up, 8, q_norm)
    code = np.minimum(((e_n + 7) << 3) | (q_n.astype(np.int64) - 8), 0x7E)
    out = np.where(e < -6, q_sub.astype(np.int64), code)
    out = np.where(a >= E4M3_MAX, 0x7E, out)
    out = (out.astype(np.uint8) | sign).astype(np.uint8)
    return np.where(np.isnan(x), np.uint8(0x7F), out).astype(np.uint8)


def e4m3_value(bits):
    """float32 values of uint8 E4M3 patterns."""
    b = np.asarray(bits, dtype=np.uint8).astype(np.int64)
    e, m = (b >> 3) & 15, b & 7
    v = np.where(e == 0, np.ldexp(m.astype(np.float64), -9), np.ldexp((8 + m).astype(np.float64), e - 10))
    v = np.where((e == 15) & (m == 7), np.nan, v)
    return np.where(b & 0x80, -v, v).astype(np.float32)


def fp8_column_scales(A):
    """(s, inv) per column of float32 A (rows x cols), as defined above."""
    A = np.asarray(A, dtype=np.float32)
    amax = np.max(np.abs(A), axis=0) if A.shape[0] else np.zeros(A.shape[1], np.float32)
    nz = amax > 0
    with np.errstate(divide="ignore"):
        s = np.where(nz, amax / np.float32(E4M3_MAX), np.float32(1.0)).astype(np.float32)
        inv = np.where(nz, np.float32(E4M3_MAX) / amax, np.float32(1.0)).astype(np.float32)
    return s, inv


def quantize_fp8(A):
    """Column-scaled FP8 form of float32 A: (Aq uint8, s float32)."""
    A = np.asarray(A, dtype=np.float32)
    s, inv = fp8_column_scales(A)
    return e4m3_bits(A * inv[None, :]), s


def dequantize_fp8(Aq, s):
    """The matrix Aq diag(s) in float64."""
    return e4m3_value(Aq).astype(np.float64) * np.asarray(s, np.float64)[None, :]


def quantize_bf16(A):
    return bf16_bits(A)


def dequantize_bf16(bits):
    return bf16_value(bits).astype(np.float64)


def operand_fp8(X, row_scale=None):
    """The FP8 skinny operand of a product: (Xq uint8, t float32) with
    X' = fl32(row_scale_j X_j) when a row scale is given."""
    X = np.asarray(X, dtype=np.float32)
    if row_scale is not None:
        X = (np.asarray(row_scale, np.float32)[:, None] * X).astype(np.float32)
    return quantize_fp8(X)


__all__ = ["bf16_bits", "bf16_value", "e4m3_bits", "e4m3_value", "fp8_column_scales", "quantize_fp8",
           "dequantize_fp8", "quantize_bf16", "dequantize_bf16", "operand_fp8"]
