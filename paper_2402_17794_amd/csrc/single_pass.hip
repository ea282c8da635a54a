// Stage 2 of the single-pass Algorithms 5 and 6 (Section 3.4): everything
// after the sketches works on l-column panels and l x l matrices in FP64.
//
//   cross        X^T Z for two tall panels (FP64 MFMA, chunk partials summed
//                in chunk order): the projections Q^T [Y | Omega] of
//                eqs. (3.13) and (3.15)-(3.16).
//   small_gemm   dense FP64 products of the small matrices, with an optional
//                elementwise division by (a_i^2 + b_j^2) for the Sylvester
//                solve of Algorithm 6.
//   gj_solve     C from C (Q^T Omega) = Q^T Y (Algorithm 5 step 4) by
//                Gauss-Jordan elimination with partial pivoting on the
//                transposed system, one workgroup, the augmented matrix in
//                registers.
//   sym_pack     the symmetric part of C shifted to positive definite,
//                in the tile layout the Cholesky kernel reads.
//   eig_finish   eigenvalues from the shifted factorisation, reordered by
//                magnitude (Algorithm 5 step 5), and the lift matrix of
//                step 6.
#include <algorithm>

#include "../../include/rsvd.h"
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

// ---------------------------------------------------------------- cross --
// Partial tiles of X^T Z (X rows x LX, Z rows x LZ, both of dtype T, FP64
// accumulation) over row chunks: one workgroup of 16 wavefronts per
// (16 x 16 output tile, chunk), rows dealt to the wavefronts 4 at a time.
constexpr int kCrossWaves = 16;

int cross_chunks(int64_t rows) { return (int)std::min<int64_t>(8, std::max<int64_t>(1, ceil_div(rows, 1024))); }
size_t cross_partials_elems(int64_t rows, int LX, int LZ) {
    return (size_t)cross_chunks(rows) * (size_t)(LX / 16) * (size_t)(LZ / 16) * 256;
}

template <typename T>
__global__ __launch_bounds__(64 * kCrossWaves) void cross_kernel(const T* __restrict__ X, int64_t ldx,
                                                                 const T* __restrict__ Z, int64_t ldz, int64_t rows,
                                                                 int LX, int LZ, int nchunks,
                                                                 double* __restrict__ part) {
    const int ntx = LX / 16, ntz = LZ / 16;
    const int ntiles = ntx * ntz;
    const int tile = blockIdx.x % ntiles;
    const int chunk = blockIdx.x / ntiles;
    const int a = tile / ntz, b = tile % ntz;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t per = round_up(ceil_div(rows, nchunks), 16);
    const int64_t r0 = (int64_t)chunk * per;
    const int64_t r1 = min<int64_t>(rows, r0 + per);
    const T* __restrict__ xa = X + a * 16 + li;
    const T* __restrict__ zb = Z + b * 16 + li;
    doublex4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    constexpr int UNR = 8;
    constexpr int STEP = 4 * kCrossWaves;
    for (int64_t k0 = r0 + 4 * wave; k0 < r1; k0 += STEP * UNR) {
        double va[UNR], vb[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t row = k0 + STEP * u + lk;
            const bool ok = row < r1;
            va[u] = ok ? (double)xa[row * ldx] : 0.0;
            vb[u] = ok ? (double)zb[row * ldz] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UNR; u += 2) {
            acc0 = mfma16x16x4(va[u], vb[u], acc0);
            acc1 = mfma16x16x4(va[u + 1], vb[u + 1], acc1);
        }
    }
    __shared__ double red[kCrossWaves][256];
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][acc_row<double>(lk, v) * 16 + li] = acc0[v] + acc1[v];
    __syncthreads();
    if (tid < 256) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < kCrossWaves; ++w) sum += red[w][tid];
        part[((size_t)chunk * ntiles + tile) * 256 + tid] = sum;
    }
}

// out (LX x LZ, ld ldo) = sum of the chunk partials in chunk order.
__global__ void cross_reduce_kernel(const double* __restrict__ part, int LX, int LZ, int nchunks,
                                    double* __restrict__ out, int ldo) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)LX * LZ) return;
    const int i = (int)(idx / LZ), j = (int)(idx % LZ);
    const int ntz = LZ / 16, ntiles = (LX / 16) * ntz;
    const int tile = (i / 16) * ntz + j / 16;
    const int e = (i % 16) * 16 + (j % 16);
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[((size_t)c * ntiles + tile) * 256 + e];
    out[(int64_t)i * ldo + j] = s;
}

hipError_t launch_cross(int dtype, const void* X, int64_t ldx, const void* Z, int64_t ldz, int64_t rows, int LX,
                        int LZ, double* partials, double* out, int ldo, hipStream_t s) {
    if (LX % 16 || LZ % 16 || LX <= 0 || LZ <= 0) return hipErrorInvalidValue;
    const int nchunks = cross_chunks(rows);
    dim3 grid(nchunks * (LX / 16) * (LZ / 16));
    if (dtype == 0)
        hipLaunchKernelGGL(cross_kernel<double>, grid, dim3(64 * kCrossWaves), 0, s, (const double*)X, ldx,
                           (const double*)Z, ldz, rows, LX, LZ, nchunks, partials);
    else
        hipLaunchKernelGGL(cross_kernel<float>, grid, dim3(64 * kCrossWaves), 0, s, (const float*)X, ldx,
                           (const float*)Z, ldz, rows, LX, LZ, nchunks, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cross_reduce_kernel, dim3((unsigned)ceil_div((int64_t)LX * LZ, 256)), dim3(256), 0, s,
                       partials, LX, LZ, nchunks, out, ldo);
    return hipGetLastError();
}

// ----------------------------------------------------------- small_gemm --
// C[i][j] (i < Mw, j < Nw) = (op(A) op(B))[i][j] for i < M, j < N, else 0;
// op(A) = A (M x K, lda) or A^T (ta), op(B) likewise.  With dr, dc given,
// C[i][j] /= dr[i]^2 + dc[j]^2.  16 x 16 outputs per workgroup, K in steps
// of 16 through LDS.
__global__ __launch_bounds__(256) void small_gemm_kernel(int M, int N, int K, const double* __restrict__ A, int lda,
                                                         int ta, const double* __restrict__ B, int ldb, int tb,
                                                         double* __restrict__ C, int ldc, int Mw, int Nw,
                                                         const double* __restrict__ dr,
                                                         const double* __restrict__ dc) {
    __shared__ double As[16][17], Bs[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
    double acc = 0.0;
    for (int k0 = 0; k0 < K; k0 += 16) {
        {
            const int ai = blockIdx.y * 16 + ty, ak = k0 + tx;         // op(A)[ai][ak]
            double v = 0.0;
            if (ai < M && ak < K) v = ta ? A[(int64_t)ak * lda + ai] : A[(int64_t)ai * lda + ak];
            As[ty][tx] = v;
            const int bk = k0 + ty, bj = blockIdx.x * 16 + tx;         // op(B)[bk][bj]
            double w = 0.0;
            if (bk < K && bj < N) w = tb ? B[(int64_t)bj * ldb + bk] : B[(int64_t)bk * ldb + bj];
            Bs[ty][tx] = w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) acc = fma(As[ty][kk], Bs[kk][tx], acc);
        __syncthreads();
    }
    if (i >= Mw || j >= Nw) return;
    double v = (i < M && j < N) ? acc : 0.0;
    if (dr && i < M && j < N) v /= dr[i] * dr[i] + dc[j] * dc[j];
    C[(int64_t)i * ldc + j] = v;
}

hipError_t launch_small_gemm(int M, int N, int K, const double* A, int lda, int ta, const double* B, int ldb, int tb,
                             double* C, int ldc, int Mw, int Nw, hipStream_t s, const double* dr,
                             const double* dc) {
    if (Mw < M || Nw < N || Mw <= 0 || Nw <= 0) return hipErrorInvalidValue;
    dim3 grid((unsigned)ceil_div(Nw, 16), (unsigned)ceil_div(Mw, 16));
    hipLaunchKernelGGL(small_gemm_kernel, grid, dim3(256), 0, s, M, N, K, A, lda, ta, B, ldb, tb, C, ldc, Mw, Nw, dr,
                       dc);
    return hipGetLastError();
}

// ------------------------------------------------------------- gj_solve --
// Solve W^T X = Z^T for X (l x l), i.e. X = C^T with C W = Z.  The
// augmented matrix [W^T | Z^T] (l x 2l) lives in registers: wavefront w
// holds columns w, w + 8, ... and lane t rows t, t + 64.  Step j: every
// wavefront reads column j from LDS (published by its owner at the end of
// step j - 1), picks the pivot p = argmax |a_rj| over the rows not yet used
// (lowest row on ties), takes row p of its own columns from the owning lane,
// normalises row p and eliminates column j from every other row.  After l
// steps the row chosen at step j holds x_j in its right half.  One barrier
// per step (the column buffer alternates).  A zero pivot sets
// RSVD_INFO_SINGULAR_SYSTEM and leaves X undefined.
constexpr int kGjWaves = 8;

__device__ __forceinline__ double readlane_f64(double x, int src) {
    int2 v = __builtin_bit_cast(int2, x);
    v.x = __builtin_amdgcn_readlane(v.x, src);
    v.y = __builtin_amdgcn_readlane(v.y, src);
    return __builtin_bit_cast(double, v);
}

template <int LT>
__global__ __launch_bounds__(64 * kGjWaves) void gj_solve_kernel(const double* __restrict__ Wt,
                                                                 const double* __restrict__ Zt, int ld, int l,
                                                                 double* __restrict__ X, int ldx, DevFlags* flags) {
    constexpr int L = 16 * LT, NR = (L + 63) / 64, NC = (2 * L + kGjWaves - 1) / kGjWaves;
    __shared__ double colbuf[2][L];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double M[NR][NC];
    bool used[NR];
    int step_of[NR];
#pragma unroll
    for (int ri = 0; ri < NR; ++ri) {
        const int r = lane + 64 * ri;
        used[ri] = r >= l;
        step_of[ri] = -1;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            const int c = w + kGjWaves * cc;
            double v = 0.0;
            if (r < l && c < 2 * l) v = c < l ? Wt[(int64_t)r * ld + c] : Zt[(int64_t)r * ld + (c - l)];
            M[ri][cc] = v;
        }
    }
    if (w == 0) {
#pragma unroll
        for (int ri = 0; ri < NR; ++ri) {
            const int r = lane + 64 * ri;
            if (r < l) colbuf[0][r] = M[ri][0];
        }
    }
    __syncthreads();
    bool singular = false;
    for (int j = 0; j < l; ++j) {
        const double* col = colbuf[j & 1];
        // Pivot search (the same in every wavefront).
        double best = -1.0;
        int bi = 1 << 30;
        double f[NR];
#pragma unroll
        for (int ri = 0; ri < NR; ++ri) {
            const int r = lane + 64 * ri;
            f[ri] = r < l ? col[r] : 0.0;
            const double a = fabs(f[ri]);
            if (!used[ri] && (a > best || (a == best && r < bi))) { best = a; bi = r; }
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double ob = __shfl_xor(best, off);
            const int oi = __shfl_xor(bi, off);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const int p = __builtin_amdgcn_readfirstlane(bi);
        if (p >= l || !(best > 0.0)) {          // no usable pivot (zero or NaN column)
            singular = true;
            break;
        }
        const int pl = p & 63, pr = p >> 6;
        const double inv = 1.0 / col[p];
#pragma unroll
        for (int ri = 0; ri < NR; ++ri)
            if (lane == pl && ri == pr) { used[ri] = true; step_of[ri] = j; }
        const int nj = j + 1;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            const double prow = readlane_f64(pr == 0 ? M[0][cc] : M[NR - 1][cc], pl) * inv;
            const int c = w + kGjWaves * cc;
#pragma unroll
            for (int ri = 0; ri < NR; ++ri) {
                const bool is_p = lane == pl && ri == pr;
                M[ri][cc] = is_p ? prow : fma(-f[ri], prow, M[ri][cc]);
                if (c == nj && nj < l) {
                    const int r = lane + 64 * ri;
                    if (r < l) colbuf[nj & 1][r] = M[ri][cc];
                }
            }
        }
        __syncthreads();
    }
    if (singular) {
        if (threadIdx.x == 0) atomicOr(&flags->info, RSVD_INFO_SINGULAR_SYSTEM);
        return;
    }
    // Row chosen at step j holds x_j (columns l .. 2l - 1).
#pragma unroll
    for (int ri = 0; ri < NR; ++ri) {
        if (step_of[ri] < 0) continue;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            const int c = w + kGjWaves * cc;
            if (c >= l && c < 2 * l) X[(int64_t)step_of[ri] * ldx + (c - l)] = M[ri][cc];
        }
    }
}

hipError_t launch_gj_solve(const double* Wt, const double* Zt, int ld, int l, double* X, int ldx, DevFlags* flags,
                           hipStream_t s) {
    const int LT = (int)ceil_div(l, 16);
#define RSVD_GJ_CASE(N)                                                                                       \
    case N:                                                                                                   \
        hipLaunchKernelGGL(gj_solve_kernel<N>, dim3(1), dim3(64 * kGjWaves), 0, s, Wt, Zt, ld, l, X, ldx, flags); \
        break;
    switch (LT) {
        RSVD_GJ_CASE(1) RSVD_GJ_CASE(2) RSVD_GJ_CASE(3) RSVD_GJ_CASE(4)
        RSVD_GJ_CASE(5) RSVD_GJ_CASE(6) RSVD_GJ_CASE(7) RSVD_GJ_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef RSVD_GJ_CASE
    return hipGetLastError();
}

// ------------------------------------------------------------- sym_pack --
// Cs = (X + X^T) / 2 for the l x l X (Cs is also the symmetric part of
// C = X^T); shift s = 2 ||Cs||_F (1 if Cs = 0), so that Cs + s I has its
// eigenvalues in [||Cs||_F, 3 ||Cs||_F]; writes Cs + s I as one chunk of
// Gram partials (16 x 16 tiles on and above the diagonal, zero outside
// l x l) and s to *shift.
__global__ __launch_bounds__(256) void sym_pack_kernel(const double* __restrict__ X, int ldx, int l, int L,
                                                       double* __restrict__ part, double* __restrict__ shift) {
    __shared__ double red[4];
    double ss = 0.0;
    for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
        const int i = idx / l, j = idx % l;
        const double c = 0.5 * (X[(int64_t)i * ldx + j] + X[(int64_t)j * ldx + i]);
        ss = fma(c, c, ss);
    }
    const double fro = sqrt(block_sum(ss, red));
    const double sh = fro > 0.0 ? 2.0 * fro : 1.0;
    const int nt = L / 16;
    const int npairs = nt * (nt + 1) / 2;
    for (int idx = threadIdx.x; idx < npairs * 256; idx += blockDim.x) {
        const int pair = idx / 256, e = idx % 256;
        int a = 0, p = pair;
        while (p >= nt - a) { p -= nt - a; ++a; }
        const int b = a + p;
        const int i = 16 * a + e / 16, j = 16 * b + e % 16;
        double v = 0.0;
        if (i < l && j < l) v = 0.5 * (X[(int64_t)i * ldx + j] + X[(int64_t)j * ldx + i]) + (i == j ? sh : 0.0);
        part[idx] = v;
    }
    if (threadIdx.x == 0) *shift = sh;
}

hipError_t launch_sym_pack(const double* X, int ldx, int l, int L, double* partials, double* shift, hipStream_t s) {
    hipLaunchKernelGGL(sym_pack_kernel, dim3(1), dim3(256), 0, s, X, ldx, l, L, partials, shift);
    return hipGetLastError();
}

// ----------------------------------------------------------- eig_finish --
// sigma, Ut: the small SVD of the Cholesky factor of Cs + s I (sigma_i^2 =
// its eigenvalues, descending; Ut's columns the eigenvectors).  Eigenvalues
// of Cs: lambda_i = sigma_i^2 - s.  Keep the k of largest |lambda| (ties:
// larger lambda, then lower index) in that order: lam_out[0..k) and the
// columns of Wu (L x ldw, zero past column k).
__global__ __launch_bounds__(256) void eig_finish_kernel(const double* __restrict__ sigma,
                                                         const double* __restrict__ Ut, int l, int L,
                                                         const double* __restrict__ shift, int k,
                                                         double* __restrict__ lam_out, double* __restrict__ Wu,
                                                         int ldw) {
    __shared__ double lam[kMaxL];
    __shared__ int slot[kMaxL];
    const double sh = *shift;
    for (int i = threadIdx.x; i < l; i += blockDim.x) lam[i] = sigma[i] * sigma[i] - sh;
    __syncthreads();
    for (int i = threadIdx.x; i < l; i += blockDim.x) {
        const double ai = fabs(lam[i]);
        int rank = 0;
        for (int j = 0; j < l; ++j) {
            const double aj = fabs(lam[j]);
            rank += (aj > ai) || (aj == ai && (lam[j] > lam[i] || (lam[j] == lam[i] && j < i)));
        }
        slot[i] = rank;
        if (rank < k) lam_out[rank] = lam[i];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < L * ldw; idx += blockDim.x) Wu[idx] = 0.0;
    __syncthreads();
    for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
        const int row = idx / l, i = idx % l;
        const int rk = slot[i];
        if (rk < k) Wu[(int64_t)row * ldw + rk] = Ut[(int64_t)row * L + i];
    }
}

hipError_t launch_eig_finish(const double* sigma, const double* Ut, int l, int L, const double* shift, int k,
                             double* lam_out, double* Wu, int ldw, hipStream_t s) {
    if (l > kMaxL || k > l || ldw < k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(eig_finish_kernel, dim3(1), dim3(256), 0, s, sigma, Ut, l, L, shift, k, lam_out, Wu, ldw);
    return hipGetLastError();
}

}  // namespace rsvd
