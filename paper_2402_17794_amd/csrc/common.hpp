// Shared device helpers for the gfx950 randomized-SVD kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

constexpr int kWave = 64;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA accumulator types: 4 values per lane.
template <typename T> struct Acc4;
template <> struct Acc4<float> { using type = floatx4; };
template <> struct Acc4<double> { using type = doublex4; };

// D(16x16) += A(16x4) B(4x16).  Operand layout per lane (64 lanes):
//   a = A[lane % 16][lane / 16],  b = B[lane / 16][lane % 16],
//   d[v] = D[acc_row<T>(lane / 16, v)][lane % 16]
// with rows 4 * (lane / 16) + v for FP32 and (lane / 16) + 4 v for FP64.
template <typename T> __device__ __forceinline__ int acc_row(int lk, int v);
template <> __device__ __forceinline__ int acc_row<float>(int lk, int v) { return 4 * lk + v; }
template <> __device__ __forceinline__ int acc_row<double>(int lk, int v) { return lk + 4 * v; }
__device__ __forceinline__ floatx4 mfma16x16x4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16x16x4(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Sum over the 16 lanes of each quarter-wave, result in all 16 lanes.
// Butterfly with DPP lane swaps: xor 1, xor 2 (quad permutes), then the
// half-row and row mirrors (i <-> 7 - i, i <-> 15 - i), which pair every
// quad with another quad and every 8-lane half with the other half.
__device__ __forceinline__ int dpp_quad_xor1(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_quad_xor2(int v) { return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_half_mirror(int v) { return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_mirror(int v) { return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true); }

template <int (*F)(int)>
__device__ __forceinline__ double dpp_f64(double x) {
    int2 v = __builtin_bit_cast(int2, x);
    v.x = F(v.x);
    v.y = F(v.y);
    return __builtin_bit_cast(double, v);
}

__device__ __forceinline__ double quarter_sum(double x) {
    x += dpp_f64<dpp_quad_xor1>(x);
    x += dpp_f64<dpp_quad_xor2>(x);
    x += dpp_f64<dpp_half_mirror>(x);
    x += dpp_f64<dpp_mirror>(x);
    return x;
}

// Full 64-lane sum (result in every lane).
__device__ __forceinline__ double wave_sum(double x) {
    x = quarter_sum(x);
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    return x;
}

// Block-wide sum for blockDim.x threads; `scratch` holds one double per wave.
__device__ __forceinline__ double block_sum(double x, double* scratch) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    x = wave_sum(x);
    __syncthreads();
    if (lane == 0) scratch[wid] = x;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += scratch[w];   // same order in every thread
    return t;
}

__host__ __device__ constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ constexpr int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Workgroup ids are dealt round-robin over the 8 XCDs (XCD = id mod 8), each
// with its own L2.  Block b = xcd_block(id, n) of n blocks gives XCD x the
// contiguous eighth x of the blocks (when 8 divides n; else b = id), so a
// chain of row-blocked kernels (split-K reduce, Gram, apply, the next
// product's slice of its thin operand) reads on each XCD the rows that the
// XCD wrote, from its own L2.
__device__ __forceinline__ int64_t xcd_block(int64_t id, int64_t n) {
    return (n % 8 == 0) ? (id % 8) * (n / 8) + id / 8 : id;
}

}  // namespace rsvd
