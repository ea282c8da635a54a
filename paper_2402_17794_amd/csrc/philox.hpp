// Counter-based Gaussian test matrix for the sketch Y = A Omega.
//
// Omega (Algorithm 4 step 1) is an n x l matrix of independent standard
// normals.  Its elements are a pure function of (seed, row, column): uniform
// bits from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11: ten rounds of
// two 32x32 -> 64-bit multiplies with xor-and-permute, key bumped by two
// Weyl constants between rounds) and normals from the Box-Muller transform.
// Block (g, j, stream, 0) under key (seed) gives the four rows 4g..4g+3 of
// column j.  No element of Omega is ever stored in device memory by the
// solve; the sketch kernel evaluates it where it is consumed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

struct Philox4 {
    uint32_t x[4];
};

__host__ __device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                          uint32_t c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
    constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kMul0 * c0;
        const uint64_t p1 = (uint64_t)kMul1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    Philox4 out;
    out.x[0] = c0; out.x[1] = c1; out.x[2] = c2; out.x[3] = c3;
    return out;
}

// Box-Muller pair from two words: u1 = ((a >> 8) + 1) 2^-24 in (0, 1],
// u2 = (b >> 8) 2^-24 in [0, 1); both exact in float and double.
// FP32: the hardware transcendentals, -2 ln u1 = -2 ln 2 log2(u1) and
// sin / cos of 2 pi u2 (the instructions take their argument in turns):
// over all 2^24 values of each uniform the normals stay within 1.5e-7
// (|z| + 1) of the exact transform (the library forms: 1.3e-7), and cost a
// fraction of the library forms in the sketch kernel.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
    const float u1 = (float)((a >> 8) + 1u) * 0x1.0p-24f;
    const float u2 = (float)(b >> 8) * 0x1.0p-24f;
    const float r = __builtin_amdgcn_sqrtf(-0x1.62e430p+0f * __builtin_amdgcn_logf(u1));
    z0 = r * __builtin_amdgcn_cosf(u2);
    z1 = r * __builtin_amdgcn_sinf(u2);
}

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1) {
    const double u1 = (double)((a >> 8) + 1u) * 0x1.0p-24;
    const double u2 = (double)(b >> 8) * 0x1.0p-24;
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// The four normals Omega[4g + 0..3][j].
template <typename T>
__device__ __forceinline__ void omega_block(uint64_t seed, uint32_t stream, uint32_t g, uint32_t j,
                                            T z[4]) {
    const Philox4 w = philox4x32_10(g, j, stream, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
    box_muller(w.x[0], w.x[1], z[0], z[1]);
    box_muller(w.x[2], w.x[3], z[2], z[3]);
}

// SRFT test matrix Omega = sqrt(n / l) D F R (real form: D = diag of +-1,
// F the orthonormal DCT-II, R the sampled columns c_j).  The sign of row i is
// bit 0 of word (i mod 4) of block (i / 4, 0, 4, 0); element (i, j) is
// sqrt(2 / l) d_i cos(pi (2 i + 1) c_j / (2 n)) (sqrt(1 / l) d_i for
// c_j = 0), the cosine taken of the argument reduced exactly modulo 2 pi in
// integers: cos(2 pi ((2 i + 1) c_j mod 4n) / 4n).
constexpr uint32_t kSrftStream = 4;

__device__ __forceinline__ void srft_signs4(uint64_t seed, uint32_t g, float d[4]) {
    const Philox4 w = philox4x32_10(g, 0u, kSrftStream, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
#pragma unroll
    for (int e = 0; e < 4; ++e) d[e] = (w.x[e] & 1u) ? -1.0f : 1.0f;
}

// (2 i + 1) c mod 4n, in 32-bit arithmetic while 4n^2 < 2^32.
__device__ __forceinline__ int64_t srft_phase(int64_t i, int c, int64_t n) {
    const int64_t q = 4 * n;
    if (q * n < ((int64_t)1 << 32)) {
        const uint32_t a = (uint32_t)((2 * i + 1) % q);
        return (int64_t)((a * (uint32_t)c) % (uint32_t)q);
    }
    return (((2 * i + 1) % q) * (int64_t)c) % q;
}
__device__ __forceinline__ float srft_cos(int64_t i, int c, int64_t n, float) {
    return __builtin_amdgcn_cosf((float)srft_phase(i, c, n) / (float)(4 * n));
}
__device__ __forceinline__ double srft_cos(int64_t i, int c, int64_t n, double) {
    return cospi((double)srft_phase(i, c, n) / (double)(2 * n));
}

// The four elements Omega[4g + 0..3][j] of column j with sampled column c;
// sc0 = sqrt(1 / l), sc1 = sqrt(2 / l).
template <typename T>
__device__ __forceinline__ void srft_block(uint64_t seed, uint32_t g, int c, int64_t n, T sc0, T sc1, T z[4]) {
    float d[4];
    srft_signs4(seed, g, d);
    const T sc = c == 0 ? sc0 : sc1;
#pragma unroll
    for (int e = 0; e < 4; ++e) z[e] = sc * (T)d[e] * srft_cos(4 * (int64_t)g + e, c, n, T(0));
}

}  // namespace rsvd
