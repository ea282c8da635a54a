// Low-precision storage formats of A on gfx950: BF16 and FP8 E4M3 (the OCP
// "E4M3FN" format the gfx950 FP8 matrix instructions read: 1 sign bit, 4
// exponent bits with bias 7, 3 mantissa bits, no infinities, 0x7F/0xFF NaN,
// largest finite value 448).  Conversions from FP32 round to nearest, ties
// to even, written out here so that every bit is specified:
//   BF16: the upper half of the FP32 pattern after adding 0x7FFF plus the
//         lowest kept bit.
//   E4M3: |x| >= 448 saturates to 448 (keeping the sign), |x| < 2^-6 is
//         rounded to a multiple of 2^-9 (subnormals), otherwise to 3
//         fractional bits of its binade.
// FP8 storage of A carries per-column FP32 scales: A ~ Aq diag(s) with
// s_j = amax_j / 448 (1 for a zero column) and Aq_ij = e4m3(A_ij * (448 /
// amax_j)), the quotient and the product each rounded in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;                  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// E4M3 with round to nearest even, saturating at +-448, NaN -> 0x7f, without
// branches: in the normal range (|x| >= 2^-6) the mantissa is rounded to 3
// bits in the FP32 bit pattern (a carry moves the exponent up), below it the
// value is q 2^-9 with q = rint(512 |x|) (q = 8 is the smallest normal).
__device__ __forceinline__ uint8_t f32_to_e4m3(float x) {
    const uint32_t u = __float_as_uint(x);
    const uint32_t sign = (u >> 24) & 0x80u;
    const uint32_t a = u & 0x7fffffffu;
    const uint32_t rn = a + 0x7ffffu + ((a >> 20) & 1u);
    const int normal = (int)(rn >> 20) - (120 << 3);          // ((e + 7) << 3) | m
    const int sub = (int)rintf(__uint_as_float(a) * 512.0f);
    int code = a >= 0x3c800000u ? normal : sub;               // 2^-6
    code = code < 0x7e ? code : 0x7e;
    return a > 0x7f800000u ? (uint8_t)0x7f : (uint8_t)(sign | (uint32_t)code);
}

__device__ __forceinline__ float e4m3_to_f32(uint8_t b) {
    const int e = (b >> 3) & 15, m = b & 7;
    float v;
    if (e == 15 && m == 7) v = __uint_as_float(0x7fc00000u);
    else if (e == 0) v = ldexpf((float)m, -9);
    else v = ldexpf((float)(8 + m), e - 10);
    return (b & 0x80) ? -v : v;
}

}  // namespace rsvd
