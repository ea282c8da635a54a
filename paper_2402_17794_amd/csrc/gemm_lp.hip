// Products with a low-precision A (BF16, or FP8 E4M3 with per-column scales)
// on the gfx950 16x16x32 BF16 / FP8 matrix instructions with FP32
// accumulation, and the conversions that feed them.
//
// The skinny operand (Q, W, or the test matrix) is converted to the same
// format as A.  A prepass writes it transposed, k-contiguous (L rows of ldt
// elements, zero padded), so that both operands of the matrix instruction are
// 16-byte LDS reads of 8 consecutive k.  The test matrix of the sketch is
// still generated inside the product kernel and written to LDS in that layout.
//
// FP8 scales: A = Aq diag(s).  For Y = A X the column scales of A fold into
// the rows of X (X' = diag(s) X) before X' is quantized with its own column
// scales t; Y = (Aq Xq) diag(t).  For Z = A^T Y, Z = diag(s) (Aq^T Yq) diag(t).
// For the sketch, Omega' = diag(s) Omega is quantized with one scale
// t = 5.77 max_j s_j / 448 (|Omega| < 5.77 by the truncation of its uniform).
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "lowp.hpp"
#include "philox.hpp"

namespace rsvd {

constexpr float kOmegaBound = 5.77f;   // sqrt(-2 ln 2^-24) < 5.77
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));   // 16 bytes in registers

// ---------------------------------------------------- matrix quantizers --
// Column maxima of |A| by atomic max on the FP32 bit patterns (non-negative
// floats order like their patterns), so the result does not depend on the
// order of the workgroups.
constexpr int kAmaxRows = 64;

__global__ __launch_bounds__(256) void col_amax_kernel(const float* __restrict__ A, int64_t rows, int64_t cols,
                                                       int64_t lda, unsigned* __restrict__ amax) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.y * kAmaxRows;
    if (c >= cols) return;
    float m = 0.0f;
    const int64_t r1 = min(rows, r0 + kAmaxRows);
    for (int64_t r = r0; r < r1; ++r) m = fmaxf(m, fabsf(A[r * lda + c]));
    atomicMax(&amax[c], __float_as_uint(m));
}

__global__ void zero_u32_kernel(unsigned* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Aq_ij = e4m3(A_ij * (448 / amax_j)); amax read from the scale buffer (bits).
__global__ __launch_bounds__(256) void quant_fp8_kernel(const float* __restrict__ A, int64_t rows, int64_t cols,
                                                        int64_t lda, uint8_t* __restrict__ Q, int64_t ldq,
                                                        const unsigned* __restrict__ amax) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t per = ceil_div(cols, 4);
    if (idx >= rows * per) return;
    const int64_t r = idx / per, c0 = (idx % per) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t c = c0 + e;
        if (c < cols) {
            const float am = __uint_as_float(amax[c]);
            const float inv = am > 0.0f ? 448.0f / am : 1.0f;
            Q[r * ldq + c] = f32_to_e4m3(A[r * lda + c] * inv);
        }
    }
}

// s_j = amax_j / 448 (1 for a zero column), in place over the amax bits.
__global__ void fp8_scales_kernel(float* __restrict__ scale, int64_t cols) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    const float am = __uint_as_float(reinterpret_cast<const unsigned*>(scale)[c]);
    scale[c] = am > 0.0f ? am / 448.0f : 1.0f;
}

__global__ __launch_bounds__(256) void quant_bf16_kernel(const float* __restrict__ A, int64_t rows, int64_t cols,
                                                         int64_t lda, uint16_t* __restrict__ Q, int64_t ldq) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t per = ceil_div(cols, 4);
    if (idx >= rows * per) return;
    const int64_t r = idx / per, c0 = (idx % per) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (c0 + e < cols) Q[r * ldq + c0 + e] = f32_to_bf16(A[r * lda + c0 + e]);
}

hipError_t launch_quantize(int fmt, const float* A, int64_t rows, int64_t cols, int64_t lda, void* Q, int64_t ldq,
                           float* col_scale, hipStream_t s) {
    if (rows == 0 || cols == 0) return hipSuccess;
    const dim3 egrid((unsigned)ceil_div(rows * ceil_div(cols, 4), 256));
    if (fmt == kFmtBf16) {
        hipLaunchKernelGGL(quant_bf16_kernel, egrid, dim3(256), 0, s, A, rows, cols, lda, (uint16_t*)Q, ldq);
        return hipGetLastError();
    }
    unsigned* amax = reinterpret_cast<unsigned*>(col_scale);
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)ceil_div(cols, 256)), dim3(256), 0, s, amax, cols);
    hipLaunchKernelGGL(col_amax_kernel, dim3((unsigned)ceil_div(cols, 256), (unsigned)ceil_div(rows, kAmaxRows)),
                       dim3(256), 0, s, A, rows, cols, lda, amax);
    hipLaunchKernelGGL(quant_fp8_kernel, egrid, dim3(256), 0, s, A, rows, cols, lda, (uint8_t*)Q, ldq, amax);
    hipLaunchKernelGGL(fp8_scales_kernel, dim3((unsigned)ceil_div(cols, 256)), dim3(256), 0, s, col_scale, cols);
    return hipGetLastError();
}

// ------------------------------------------------------ operand prepass --
// Xt[c][k] = fmt(X'[k][c]) for c < ncols, k < K; zero for ncols <= c < L and
// K <= k < ldt.  FP8: X'_kc = fl32(rs_k X_kc) (rs = the row scale, or none),
// t_c = amax_c / 448, Xq = e4m3(X' * (448 / amax_c)).  Tiles of 64 k x 64
// columns go through LDS so that both the read of X and the write of Xt are
// coalesced.
__global__ __launch_bounds__(256) void x_amax_kernel(const float* __restrict__ X, int64_t K, int ncols, int64_t ldx,
                                                     const float* __restrict__ rs, unsigned* __restrict__ amax) {
    const int c = threadIdx.x & 63, kq = threadIdx.x >> 6;
    const int64_t k0 = (int64_t)blockIdx.x * 256;
    const int cc = blockIdx.y * 64 + c;
    if (cc >= ncols) return;
    float m = 0.0f;
    for (int64_t k = k0 + kq; k < min(K, k0 + 256); k += 4) {
        float v = X[k * ldx + cc];
        if (rs) v = rs[k] * v;
        m = fmaxf(m, fabsf(v));
    }
    atomicMax(&amax[cc], __float_as_uint(m));
}

template <int AB>
__global__ __launch_bounds__(256) void x_prep_kernel(const float* __restrict__ X, int64_t K, int ncols, int64_t ldx,
                                                     const float* __restrict__ rs, const unsigned* __restrict__ amax,
                                                     uint8_t* __restrict__ Xt, int64_t ldt, int L,
                                                     float* __restrict__ tsc) {
    __shared__ float tileS[64][65];
    const int tid = threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64;
    for (int i = tid; i < 64 * 64; i += 256) {
        const int kk = i >> 6, c = i & 63;
        const int64_t k = k0 + kk;
        float v = 0.0f;
        if (k < K && c0 + c < ncols) {
            v = X[k * ldx + c0 + c];
            if (rs) v = rs[k] * v;
        }
        tileS[kk][c] = v;
    }
    __syncthreads();
    for (int i = tid; i < 64 * 64; i += 256) {
        const int c = i >> 6, kk = i & 63;
        const int64_t k = k0 + kk;
        if (k >= ldt || c0 + c >= L) continue;
        const float v = tileS[kk][c];
        if (AB == 2) {
            reinterpret_cast<uint16_t*>(Xt)[(int64_t)(c0 + c) * ldt + k] = f32_to_bf16(v);
        } else {
            const float am = (c0 + c < ncols) ? __uint_as_float(amax[c0 + c]) : 0.0f;
            const float inv = am > 0.0f ? 448.0f / am : 1.0f;
            Xt[(int64_t)(c0 + c) * ldt + k] = f32_to_e4m3(v * inv);
        }
    }
    if (AB == 1 && blockIdx.x == 0 && tid < 64 && c0 + tid < ncols) {
        const float am = __uint_as_float(amax[c0 + tid]);
        tsc[c0 + tid] = am > 0.0f ? am / 448.0f : 1.0f;
    }
}

hipError_t launch_lp_operand(int fmt, const float* X, int64_t K, int ncols, int64_t ldx, const float* row_scale,
                             void* Xt, int64_t ldt, int L, float* tscale, unsigned* amax_tmp, hipStream_t s) {
    const dim3 grid((unsigned)ceil_div(ldt, 64), (unsigned)(L / 16 + 3) / 4);   // 64-column groups covering L
    if (fmt == kFmtBf16) {
        hipLaunchKernelGGL(x_prep_kernel<2>, grid, dim3(256), 0, s, X, K, ncols, ldx, (const float*)nullptr,
                           (const unsigned*)nullptr, (uint8_t*)Xt, ldt, L, (float*)nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)ceil_div(L, 256)), dim3(256), 0, s, amax_tmp, (int64_t)L);
    hipLaunchKernelGGL(x_amax_kernel, dim3((unsigned)std::max<int64_t>(1, ceil_div(K, 256)), (unsigned)ceil_div(ncols, 64)),
                       dim3(256), 0, s, X, K, ncols, ldx, row_scale, amax_tmp);
    hipLaunchKernelGGL(x_prep_kernel<1>, grid, dim3(256), 0, s, X, K, ncols, ldx, row_scale, amax_tmp,
                       (uint8_t*)Xt, ldt, L, tscale);
    return hipGetLastError();
}

// max_j s_j of the FP8 scales (one workgroup).
__global__ __launch_bounds__(256) void vec_max_kernel(const float* __restrict__ v, int64_t n, float* __restrict__ out) {
    __shared__ float red[256];
    float m = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmaxf(m, v[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t launch_vec_max(const float* v, int64_t n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(vec_max_kernel, dim3(1), dim3(256), 0, s, v, n, out);
    return hipGetLastError();
}

// -------------------------------------------------------- product kernel --
// 256 threads, BM = 128 rows of the output (wavefront w: rows 32w..32w+31, two
// 16-row tiles), all L = 16 LT columns, K tiles of 64 (two instruction steps
// of 32).  LDS: A tile (NN: [BM][64] k-contiguous; TN: [64][BM] as in memory,
// read 8 k per lane with 2-byte / 1-byte loads) and the operand tile [L][64].
// Strides padded so that the four lane groups of a fragment read hit
// different banks.
template <int AB> struct LpFrag;
template <> struct LpFrag<2> {
    using type = bf16x8;
    __device__ static floatx4 mfma(type a, type b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct LpFrag<1> {
    using type = long;
    __device__ static floatx4 mfma(type a, type b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
    }
};

template <int AB, bool TRANS, bool OMEGA, int LT>
__global__ __launch_bounds__(256) void lp_gemm_kernel(LpGemmArgs g) {
    constexpr int RT = 2, BM = 128, BK = 64, L = 16 * LT;
    constexpr int EPV = 16 / AB;                         // elements per 16-byte vector
    constexpr int ROWB = BK * AB;                        // bytes of 64 k of one row
    constexpr int SA = TRANS ? BM * AB + 8 : ROWB + 16;  // LDS row stride (bytes)
    constexpr int A_BYTES = TRANS ? BK * SA : BM * SA;
    constexpr int SX = ROWB + 16;
    constexpr int NVA = BM * ROWB / 16 / 256;            // A vectors per thread
    constexpr int NVX = (L * ROWB / 16 + 255) / 256;     // operand vectors per thread
    constexpr int NOB = (L * (BK / 4) + 255) / 256;      // test-matrix blocks per thread
    using F = LpFrag<AB>;
    using FT = typename F::type;

    __shared__ __attribute__((aligned(16))) uint8_t As[A_BYTES];
    __shared__ __attribute__((aligned(16))) uint8_t Xs[L * SX];

    const uint8_t* __restrict__ A = static_cast<const uint8_t*>(g.A);
    const uint8_t* __restrict__ Xt = static_cast<const uint8_t*>(g.Xt);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int split = blockIdx.x % g.splits, tile = blockIdx.x / g.splits;
    const int64_t row0 = (int64_t)tile * BM;
    const int64_t kchunk = round_up(ceil_div(g.K, g.splits), BK);
    const int64_t kbeg = (int64_t)split * kchunk;
    const int64_t kend = min(g.K, kbeg + kchunk);

    floatx4 acc[RT][LT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < LT; ++t) acc[r][t] = floatx4{0, 0, 0, 0};

    u32x4 ra[NVA];
    u32x4 rx[OMEGA ? 1 : NVX];
    const bool rows_full = row0 + BM <= g.M;
    // A: NN rows row0.., k columns; TN k rows, columns row0..  Vectors wholly
    // inside A take one 16-byte load; the edges go element by element.
    auto load_a = [&](int64_t k0) {
        const bool full = rows_full && k0 + BK <= kend;
#pragma unroll
        for (int it = 0; it < NVA; ++it) {
            const int idx = tid + 256 * it;
            int64_t row, col;                            // element (row, col) of A in memory
            if (!TRANS) { row = row0 + idx / (ROWB / 16); col = k0 + (idx % (ROWB / 16)) * EPV; }
            else        { row = k0 + idx / (BM * AB / 16); col = row0 + (idx % (BM * AB / 16)) * EPV; }
            const int64_t rlim = TRANS ? kend : g.M, clim = TRANS ? g.M : kend;
            if (full || (row < rlim && col + EPV <= clim)) {
                ra[it] = *reinterpret_cast<const u32x4*>(A + (row * g.lda + col) * AB);
            } else {
                uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int64_t ce = col + e / AB;
                    const uint32_t byte = (row < rlim && ce < clim) ? A[(row * g.lda + ce) * AB + e % AB] : 0u;
                    w[e >> 2] |= byte << (8 * (e & 3));
                }
                ra[it] = u32x4{w[0], w[1], w[2], w[3]};
            }
        }
    };
    auto store_a = [&]() {
#pragma unroll
        for (int it = 0; it < NVA; ++it) {
            const int idx = tid + 256 * it;
            int off;
            if (!TRANS) off = (idx / (ROWB / 16)) * SA + (idx % (ROWB / 16)) * 16;
            else        off = (idx / (BM * AB / 16)) * SA + (idx % (BM * AB / 16)) * 16;
            if (TRANS) {     // SA is a multiple of 8, not 16, in this layout: two 8-byte stores
                *reinterpret_cast<uint2*>(&As[off]) = make_uint2(ra[it].x, ra[it].y);
                *reinterpret_cast<uint2*>(&As[off + 8]) = make_uint2(ra[it].z, ra[it].w);
            } else {
                *reinterpret_cast<u32x4*>(&As[off]) = ra[it];
            }
        }
    };
    // Operand: L rows of the prepared Xt (zero padded: always in bounds).
    auto load_x = [&](int64_t k0) {
        if constexpr (!OMEGA) {
#pragma unroll
            for (int it = 0; it < NVX; ++it) {
                // the index is clamped so that every thread loads (the surplus is never stored)
                const int idx = min(tid + 256 * it, L * ROWB / 16 - 1);
                const int c = idx / (ROWB / 16), kb = (idx % (ROWB / 16)) * EPV;
                rx[it] = *reinterpret_cast<const u32x4*>(Xt + ((int64_t)c * g.ldt + k0 + kb) * AB);
            }
        }
    };
    auto store_x = [&](int64_t k0) {
        if constexpr (OMEGA) {
            // Omega'_kj for rows k0 + 4 gi .. + 3 of column j, FP8: diag(s) Omega / t.
            float inv_t = 1.0f, sk[4] = {0.f, 0.f, 0.f, 0.f};
            static_assert(256 % (BK / 4) == 0, "a thread keeps its 4 rows of k");
            if (AB == 1) {
                inv_t = 448.0f / (kOmegaBound * g.omega_scale[0]);
                const int64_t r = k0 + 4 * (tid % (BK / 4));
#pragma unroll
                for (int e = 0; e < 4; ++e) sk[e] = r + e < kend ? g.col_scale[r + e] : 0.f;
            }
#pragma unroll
            for (int it = 0; it < NOB; ++it) {
                const int idx = tid + 256 * it;
                if (idx < L * (BK / 4)) {
                    const int j = idx / (BK / 4), gi = idx % (BK / 4);
                    const int64_t r = k0 + 4 * gi;
                    float z[4] = {0.f, 0.f, 0.f, 0.f};
                    if (j < g.ncols && r < kend) omega_block<float>(g.seed, 0u, (uint32_t)(r >> 2), (uint32_t)j, z);
                    uint8_t* dst = &Xs[j * SX + 4 * gi * AB];
                    if (AB == 2) {
                        uint16_t h[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) h[e] = f32_to_bf16(r + e < kend ? z[e] : 0.f);
                        *reinterpret_cast<uint2*>(dst) = make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
                    } else {
                        uint32_t w = 0;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float v = (r + e < kend) ? (sk[e] * z[e]) * inv_t : 0.f;
                            w |= (uint32_t)f32_to_e4m3(v) << (8 * e);
                        }
                        *reinterpret_cast<uint32_t*>(dst) = w;
                    }
                }
            }
        } else {
#pragma unroll
            for (int it = 0; it < NVX; ++it) {
                const int idx = tid + 256 * it;
                if (idx < L * ROWB / 16) {
                    const int c = idx / (ROWB / 16), kb = (idx % (ROWB / 16)) * 16;
                    *reinterpret_cast<u32x4*>(&Xs[c * SX + kb]) = rx[it];
                }
            }
            (void)k0;
        }
    };

    const int wm = wave * 32;
    const int li = lane & 15, lk = lane >> 4;
    if (kbeg < kend) {
        load_a(kbeg);
        load_x(kbeg);
        for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
            __syncthreads();
            store_a();
            store_x(k0);
            __syncthreads();
            if (k0 + BK < kend) {
                load_a(k0 + BK);
                load_x(k0 + BK);
            }
#pragma unroll
            for (int kk = 0; kk < BK; kk += 32) {
                FT fa[RT], fx[LT];
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    if (!TRANS) {
                        fa[r] = *reinterpret_cast<const FT*>(&As[(wm + 16 * r + li) * SA + (kk + 8 * lk) * AB]);
                    } else if constexpr (AB == 2) {
                        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const uint32_t h =
                                *reinterpret_cast<const uint16_t*>(&As[(kk + 8 * lk + i) * SA + (wm + 16 * r + li) * 2]);
                            w[i >> 1] |= h << (16 * (i & 1));
                        }
                        fa[r] = __builtin_bit_cast(FT, u32x4{w[0], w[1], w[2], w[3]});
                    } else {
                        uint32_t w[2] = {0u, 0u};
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const uint32_t b = As[(kk + 8 * lk + i) * SA + wm + 16 * r + li];
                            w[i >> 2] |= b << (8 * (i & 3));
                        }
                        fa[r] = __builtin_bit_cast(FT, ((uint64_t)w[1] << 32) | w[0]);
                    }
                }
#pragma unroll
                for (int t = 0; t < LT; ++t)
                    fx[t] = *reinterpret_cast<const FT*>(&Xs[(16 * t + li) * SX + (kk + 8 * lk) * AB]);
#pragma unroll
                for (int t = 0; t < LT; ++t)
#pragma unroll
                    for (int r = 0; r < RT; ++r) acc[r][t] = F::mfma(fa[r], fx[t], acc[r][t]);
            }
        }
    }

    // Epilogue: scales (FP8), then Y or the split-K slice.
    const int64_t pstride = g.M * L;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < LT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + wm + 16 * r + 4 * lk + v;
                const int col = 16 * t + li;
                if (row >= g.M) continue;
                float y = acc[r][t][v];
                if (AB == 1) {
                    if (TRANS) y *= g.col_scale[row];
                    if (OMEGA) y *= kOmegaBound * g.omega_scale[0] / 448.0f;
                    else if (col < g.ncols) y *= g.xscale[col];
                }
                if (g.splits == 1) {
                    if (col < g.wcols) g.Y[row * g.ldy + col] = y;
                } else {
                    g.partials[split * pstride + row * L + col] = y;
                }
            }
}

static int lp_row_tiles(int64_t M) { return (int)ceil_div(M, 128); }

static int lp_choose_splits(int64_t M, int64_t K) {
    const int tiles = lp_row_tiles(M);
    const int64_t ktiles = ceil_div(K, 64);
    int s = (int)ceil_div(512, tiles);
    s = (int)std::min<int64_t>(s, std::max<int64_t>(1, ktiles / 8));
    return std::max(1, std::min(s, kMaxSplits));
}

size_t lp_partials_elems(int64_t M, int64_t K, int ncols, int* splits_out) {
    const int s = lp_choose_splits(M, K);
    if (splits_out) *splits_out = s;
    return s > 1 ? (size_t)s * (size_t)M * (size_t)round_up(ncols, 16) : 0;
}

template <int AB, bool TRANS, bool OMEGA>
static hipError_t lp_dispatch(const LpGemmArgs& a, int LT, dim3 grid, hipStream_t s) {
#define RSVD_LP_CASE(N) \
    case N: hipLaunchKernelGGL((lp_gemm_kernel<AB, TRANS, OMEGA, N>), grid, dim3(256), 0, s, a); break;
    switch (LT) {
        RSVD_LP_CASE(1) RSVD_LP_CASE(2) RSVD_LP_CASE(3) RSVD_LP_CASE(4) RSVD_LP_CASE(5) RSVD_LP_CASE(6)
        RSVD_LP_CASE(7) RSVD_LP_CASE(8) RSVD_LP_CASE(9) RSVD_LP_CASE(10) RSVD_LP_CASE(11) RSVD_LP_CASE(12)
        RSVD_LP_CASE(13) RSVD_LP_CASE(14) RSVD_LP_CASE(15) RSVD_LP_CASE(16) RSVD_LP_CASE(17) RSVD_LP_CASE(18)
        default: return hipErrorInvalidValue;
    }
#undef RSVD_LP_CASE
    return hipGetLastError();
}

hipError_t launch_lp_gemm(int fmt, LpGemmArgs a, hipStream_t s, hipEvent_t product_done) {
    if (a.ncols < 1 || a.ncols > kMaxL || a.M < 0 || a.K < 0) return hipErrorInvalidValue;
    if (a.M == 0) return product_done ? hipEventRecord(product_done, s) : hipSuccess;
    const int LT = (int)ceil_div(a.ncols, 16);
    const bool omega = a.Xt == nullptr;
    if (omega && a.trans) return hipErrorInvalidValue;
    if (a.splits < 1 || a.splits > kMaxSplits) return hipErrorInvalidValue;
    const dim3 grid(lp_row_tiles(a.M) * a.splits);
    hipError_t e;
    if (fmt == kFmtBf16) {
        if (a.trans) e = lp_dispatch<2, true, false>(a, LT, grid, s);
        else e = omega ? lp_dispatch<2, false, true>(a, LT, grid, s) : lp_dispatch<2, false, false>(a, LT, grid, s);
    } else {
        if (a.trans) e = lp_dispatch<1, true, false>(a, LT, grid, s);
        else e = omega ? lp_dispatch<1, false, true>(a, LT, grid, s) : lp_dispatch<1, false, false>(a, LT, grid, s);
    }
    if (e == hipSuccess && product_done) e = hipEventRecord(product_done, s);
    if (e != hipSuccess || a.splits == 1) return e;
    return launch_splitk_reduce_f32(a.partials, a.M, 16 * LT, a.splits, a.Y, a.ldy, a.wcols, s);
}

}  // namespace rsvd
