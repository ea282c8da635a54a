// Stage 2 of Algorithm 4 on gfx950: the SVD of the small matrix B = Q^T A
// (step 7), the lift U = Q U~ (step 8), truncation and signs.
//
// B is l x n with l << n; the kernels hold B^T (n x l, produced by the same
// A^T X product as the power loop).  Its Gram matrix G = B B^T (l x l, FP64)
// is factored G = R^T R, and the one-sided (Hestenes) Jacobi iteration is run
// on X = R^T: plane rotations on the right of X until its columns are
// mutually orthogonal.  Then X = U' Sigma J^T with R^T R = U' Sigma^2 U'^T =
// B B^T, so the normalised columns U' are the left singular vectors U~ of B
// and the column norms its singular values; the right singular vectors are
// V = B^T U~ Sigma^{-1}.  Neither the rotations nor R^{-1} are needed.
//
// The Jacobi runs in one workgroup of 16 wavefronts: each round of the
// round-robin ordering pairs all columns disjointly, and each quarter-wave
// (16 lanes) takes one pair, forming the three inner products with DPP lane
// sums (no LDS traffic, no barrier) before rotating the two columns in LDS.
// One barrier per round.
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "../../include/rsvd.h"

namespace rsvd {

constexpr int kJacobiLdsMax = 128;
constexpr double kJacobiTol = 1e-15;
constexpr int kJacobiMaxSweeps = 60;

// Sum over the 8 lanes of each eighth of a wavefront (xor 1, xor 2, then
// lane i <-> 7 - i within each 8-lane half-row), result in all 8 lanes.
__device__ __forceinline__ double octet_sum(double x) {
    x += dpp_f64<dpp_quad_xor1>(x);
    x += dpp_f64<dpp_quad_xor2>(x);
    x += dpp_f64<dpp_half_mirror>(x);
    return x;
}

// Sum over the 4 lanes of each quad (xor 1, then xor 2), result in all 4.
__device__ __forceinline__ double quad_sum(double x) {
    x += dpp_f64<dpp_quad_xor1>(x);
    x += dpp_f64<dpp_quad_xor2>(x);
    return x;
}

template <int LPP>
__device__ __forceinline__ double group_sum(double x) {
    static_assert(LPP == 4 || LPP == 8, "lanes per pair");
    return LPP == 4 ? quad_sum(x) : octet_sum(x);
}

// Round-robin (circle method) schedule: with n2 (even) columns, round r pairs
// slot 0 with (n2 - 1, r) and slot s > 0 with ((r + s), (r - s)) mod (n2 - 1).
__device__ __forceinline__ void rr_pair(int r, int s, int n2, int& p1, int& p2) {
    const int m = n2 - 1;
    if (s == 0) { p1 = m; p2 = r; return; }
    p1 = r + s; if (p1 >= m) p1 -= m;
    p2 = r - s + m; if (p2 >= m) p2 -= m;
}

// One-sided Jacobi on X = R^T; LPP lanes per column pair.  Columns are
// stored with a padded stride (zero rows past l stay zero under rotations),
// so every lane loads and stores its rows 2e, 2e+1, 2e+2 LPP, 2e+2 LPP+1, ...
// as 16-byte pairs without bounds checks.  NP = row pairs per lane.  Both
// forms use 8 lanes per pair: with 4 (one wavefront per SIMD) a round was
// slower, the latencies no longer hidden.
template <int NP, bool IN_LDS, int NT, int LPP>
__global__ __launch_bounds__(NT) void jacobi_kernel(const double* __restrict__ R, int l, int L,
                                                      const double* __restrict__ shift_p, double* __restrict__ sigma,
                                                      double* __restrict__ Ut, double* __restrict__ Mv,
                                                      DevFlags* flags, double* __restrict__ work) {
    __shared__ __attribute__((aligned(16))) double lds[IN_LDS ? kJacobiLdsMax * kJacobiLdsMax : 2];
    __shared__ int rotated;
    __shared__ double nrm2[kMaxL];
    __shared__ int rank_of[kMaxL];
    const int ld = IN_LDS ? kJacobiLdsMax : kMaxL;  // column stride (>= 16 * NP rows)
    double* X = IN_LDS ? lds : work;                // X[c * ld + r] = R[c][r], zero for r >= l
    const int tid = threadIdx.x, grp = tid / LPP, e = tid % LPP;
    static_assert(2 * NP * LPP <= (IN_LDS ? kJacobiLdsMax : kMaxL), "rows per column");

    for (int idx = tid; idx < l * ld; idx += NT) {
        const int c = idx / ld, r = idx - c * ld;
        X[idx] = r < l ? R[(int64_t)c * L + r] : 0.0;
    }
    const int n2 = l + (l & 1);
    bool converged = (l < 2);
    __syncthreads();
    for (int sweep = 0; sweep < kJacobiMaxSweeps && !converged; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < n2 - 1; ++r) {
            for (int s = grp; s < n2 / 2; s += NT / LPP) {
                int p1, p2;
                rr_pair(r, s, n2, p1, p2);
                if (p1 >= l || p2 >= l) continue;
                const int i = min(p1, p2), j = max(p1, p2);
                double2* xi_p = reinterpret_cast<double2*>(X + i * ld) + e;
                double2* xj_p = reinterpret_cast<double2*>(X + j * ld) + e;
                double2 xi[NP], xj[NP];
                double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
                for (int t = 0; t < NP; ++t) {
                    xi[t] = xi_p[LPP * t];
                    xj[t] = xj_p[LPP * t];
                }
#pragma unroll
                for (int t = 0; t < NP; ++t) {
                    a = fma(xi[t].x, xi[t].x, a); a = fma(xi[t].y, xi[t].y, a);
                    b = fma(xj[t].x, xj[t].x, b); b = fma(xj[t].y, xj[t].y, b);
                    g = fma(xi[t].x, xj[t].x, g); g = fma(xi[t].y, xj[t].y, g);
                }
                a = group_sum<LPP>(a);
                b = group_sum<LPP>(b);
                g = group_sum<LPP>(g);
                if (fabs(g) > kJacobiTol * sqrt(a * b)) {
                    const double zeta = (b - a) / (2.0 * g);
                    const double az = fabs(zeta);
                    double t = az > 1e150 ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az));
                    t = zeta >= 0.0 ? t : -t;
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll
                    for (int u = 0; u < NP; ++u) {
                        double2 ni, nj;
                        ni.x = c * xi[u].x - sn * xj[u].x;
                        ni.y = c * xi[u].y - sn * xj[u].y;
                        nj.x = sn * xi[u].x + c * xj[u].x;
                        nj.y = sn * xi[u].y + c * xj[u].y;
                        xi_p[LPP * u] = ni;
                        xj_p[LPP * u] = nj;
                    }
                    if (e == 0) rotated = 1;
                }
            }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        converged = (any == 0);
    }
    if (!converged && tid == 0) atomicOr(&flags->info, RSVD_INFO_JACOBI_NOT_CONVERGED);

    for (int c = grp; c < l; c += NT / LPP) {
        double s2 = 0.0;
        for (int row = e; row < l; row += LPP) s2 = fma(X[c * ld + row], X[c * ld + row], s2);
        s2 = group_sum<LPP>(s2);
        if (e == 0) nrm2[c] = s2;
    }
    __syncthreads();
    const double shift = *shift_p;
    // Stable descending order of the singular values sqrt(max(nrm2 - shift, 0)).
    for (int c = tid; c < l; c += NT) {
        const double sc = sqrt(fmax(nrm2[c] - shift, 0.0));
        int rank = 0;
        for (int d = 0; d < l; ++d) {
            const double sd = sqrt(fmax(nrm2[d] - shift, 0.0));
            rank += (sd > sc) || (sd == sc && d < c);
        }
        rank_of[c] = rank;
        sigma[rank] = sc;
    }
    __syncthreads();
    for (int idx = tid; idx < L * L; idx += NT) {
        Ut[idx] = 0.0;
        Mv[idx] = 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < l * l; idx += NT) {
        const int c = idx / l, row = idx - c * l;
        const double nc = sqrt(nrm2[c]);
        const double sc = sqrt(fmax(nrm2[c] - shift, 0.0));
        const double u = nc > 0.0 ? X[c * ld + row] / nc : (row == c ? 1.0 : 0.0);
        const int col = rank_of[c];
        Ut[(int64_t)row * L + col] = u;
        Mv[(int64_t)row * L + col] = sc > 0.0 ? u / sc : 0.0;
    }
}

hipError_t launch_jacobi(const double* R, int l, int L, const double* shift, double* sigma, double* Ut, double* Mv,
                         DevFlags* flags, double* work, hipStream_t s) {
    if (l <= kJacobiLdsMax)
        hipLaunchKernelGGL((jacobi_kernel<kJacobiLdsMax / 16, true, 1024, 8>), dim3(1), dim3(1024), 0, s, R, l, L,
                           shift, sigma, Ut, Mv, flags, work);
    else
        // 36 register pairs per lane: 512 threads leave 256 VGPRs per lane.
        hipLaunchKernelGGL((jacobi_kernel<kMaxL / 16, false, 512, 8>), dim3(1), dim3(512), 0, s, R, l, L, shift,
                           sigma, Ut, Mv, flags, work);
    return hipGetLastError();
}

// Signs: for each returned column c of V, the entry of largest magnitude
// (lowest row on ties) is made positive.  One workgroup per column reduces
// the per-block partials, which are in row order.
__global__ __launch_bounds__(256) void signs_kernel(const double* __restrict__ av, const int* __restrict__ ai,
                                                   int nblocks, int r, const double* __restrict__ sigma,
                                                   double* __restrict__ S_out, double* __restrict__ sign) {
    (void)ai;
    const int c = blockIdx.x, tid = threadIdx.x;
    __shared__ double bm[256], bv[256];
    __shared__ int bb[256];
    double best = -1.0, val = 0.0;
    int bestb = 0x7fffffff;
    for (int b = tid; b < nblocks; b += 256) {      // increasing b: strict > keeps the lowest block
        const double v = av[(int64_t)b * r + c];
        if (fabs(v) > best) { best = fabs(v); val = v; bestb = b; }
    }
    bm[tid] = best; bv[tid] = val; bb[tid] = bestb;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            const double m2 = bm[tid + off];
            const int b2 = bb[tid + off];
            if (m2 > bm[tid] || (m2 == bm[tid] && b2 < bb[tid])) { bm[tid] = m2; bv[tid] = bv[tid + off]; bb[tid] = b2; }
        }
        __syncthreads();
    }
    if (tid == 0) {
        sign[c] = bv[0] < 0.0 ? -1.0 : 1.0;
        S_out[c] = sigma[c];
    }
}

hipError_t launch_signs(const double* av, const int* ai, int nblocks, int r, const double* sigma, double* S_out,
                        double* sign, hipStream_t s) {
    if (r == 0) return hipSuccess;
    hipLaunchKernelGGL(signs_kernel, dim3(r), dim3(256), 0, s, av, ai, nblocks, r, sigma, S_out, sign);
    return hipGetLastError();
}

template <typename T>
__global__ void scale_rows_kernel(T* X, int64_t ld, int rows, int64_t cols, const double* sign) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * cols) return;
    const int r = (int)(idx / cols);
    const int64_t c = idx % cols;
    if (sign[r] < 0.0) X[r * ld + c] = -X[r * ld + c];
}

hipError_t launch_scale_rows(int dtype, void* X, int64_t ld, int rows, int64_t cols, const double* sign,
                             hipStream_t s) {
    const int64_t total = (int64_t)rows * cols;
    if (total == 0) return hipSuccess;
    dim3 grid((unsigned)ceil_div(total, 256));
    if (dtype == 0) hipLaunchKernelGGL(scale_rows_kernel<double>, grid, dim3(256), 0, s, (double*)X, ld, rows, cols, sign);
    else hipLaunchKernelGGL(scale_rows_kernel<float>, grid, dim3(256), 0, s, (float*)X, ld, rows, cols, sign);
    return hipGetLastError();
}

__global__ void init_kernel(int* counters, int count, DevFlags* flags) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) counters[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 64) reinterpret_cast<int*>(flags)[threadIdx.x] = 0;
}

hipError_t launch_init(int* counters, int count, DevFlags* flags, hipStream_t s) {
    hipLaunchKernelGGL(init_kernel, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(64, ceil_div(count, 256)))), dim3(256),
                       0, s, counters, count, flags);
    return hipGetLastError();
}

__global__ void export_info_kernel(const DevFlags* flags, int* info) { *info = flags->info; }

hipError_t launch_export_info(const DevFlags* flags, int* info, hipStream_t s) {
    hipLaunchKernelGGL(export_info_kernel, dim3(1), dim3(1), 0, s, flags, info);
    return hipGetLastError();
}

template <typename T>
__global__ void copy2d_kernel(const T* src, int64_t lds, int64_t rows, int cols, T* dst, int64_t ldd, int dcols) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * dcols) return;
    const int64_t r = idx / dcols;
    const int c = (int)(idx % dcols);
    dst[r * ldd + c] = c < cols ? src[r * lds + c] : T(0);
}

hipError_t launch_copy2d(int dtype, const void* src, int64_t lds, int64_t rows, int cols, void* dst, int64_t ldd,
                         int dcols, hipStream_t s) {
    const int64_t total = rows * dcols;
    if (total == 0) return hipSuccess;
    dim3 grid((unsigned)ceil_div(total, 256));
    if (dtype == 0)
        hipLaunchKernelGGL(copy2d_kernel<double>, grid, dim3(256), 0, s, (const double*)src, lds, rows, cols,
                           (double*)dst, ldd, dcols);
    else
        hipLaunchKernelGGL(copy2d_kernel<float>, grid, dim3(256), 0, s, (const float*)src, lds, rows, cols,
                           (float*)dst, ldd, dcols);
    return hipGetLastError();
}

}  // namespace rsvd

namespace rsvd {

// ||A - Q B||_F for the error measure of Theorems 2, 3, 6 (Frobenius form):
// each workgroup forms a 64 x 64 tile of E = A - Q (B^T)^T in FP64 from the
// stored Q and B^T and writes the sum of its squares; a second kernel adds
// the tile sums in a fixed order.
constexpr int kResTile = 64;

size_t residual_partials(int64_t m, int64_t n) {
    return (size_t)ceil_div(m, kResTile) * (size_t)ceil_div(n, kResTile);
}

template <typename T>
__global__ __launch_bounds__(256) void residual_fro_kernel(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                           const T* __restrict__ Q, const T* __restrict__ Bt, int L,
                                                           double* __restrict__ part) {
    __shared__ double Qs[16][kResTile + 1];
    __shared__ double Bs[16][kResTile + 1];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const int64_t ntn = ceil_div(n, kResTile);
    const int64_t i0 = (blockIdx.x / ntn) * kResTile, j0 = (blockIdx.x % ntn) * kResTile;
    const int ti = (tid >> 4) * 4, tj = (tid & 15) * 4;
    double acc[4][4] = {};
    for (int a0 = 0; a0 < L; a0 += 16) {
        __syncthreads();
        for (int idx = tid; idx < 16 * kResTile; idx += 256) {
            const int rr = idx >> 4, aa = idx & 15;
            Qs[aa][rr] = (i0 + rr < m) ? (double)Q[(i0 + rr) * L + a0 + aa] : 0.0;
            Bs[aa][rr] = (j0 + rr < n) ? (double)Bt[(j0 + rr) * L + a0 + aa] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int aa = 0; aa < 16; ++aa)
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(Qs[aa][ti + u], Bs[aa][tj + v], acc[u][v]);
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = i0 + ti + u, j = j0 + tj + v;
            if (i < m && j < n) {
                const double e = (double)A[i * lda + j] - acc[u][v];
                s = fma(e, e, s);
            }
        }
    s = block_sum(s, red);
    if (tid == 0) part[blockIdx.x] = s;
}

// Sum of the tile partials in a fixed order (thread-strided, then the block
// sum in wave order), and the square root.
__global__ __launch_bounds__(256) void residual_final_kernel(const double* __restrict__ part, int64_t n,
                                                             double* __restrict__ out) {
    __shared__ double red[4];
    double t = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) t += part[i];
    t = block_sum(t, red);
    if (threadIdx.x == 0) {
        out[0] = 0.0;
        out[1] = sqrt(t);
    }
}

hipError_t launch_residual_fro(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, const void* Q,
                               const void* Bt, int l, int L, double* partial, double* out, hipStream_t s) {
    (void)l;
    const int64_t ntiles = (int64_t)residual_partials(m, n);
    dim3 grid((unsigned)ntiles);
    if (dtype == 0)
        hipLaunchKernelGGL(residual_fro_kernel<double>, grid, dim3(256), 0, s, (const double*)A, lda, m, n,
                           (const double*)Q, (const double*)Bt, L, partial);
    else
        hipLaunchKernelGGL(residual_fro_kernel<float>, grid, dim3(256), 0, s, (const float*)A, lda, m, n,
                           (const float*)Q, (const float*)Bt, L, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(256), 0, s, partial, ntiles, out);
    return hipGetLastError();
}

}  // namespace rsvd

namespace rsvd {

// Spectral norm of E = A - Q Q^T A by block power iteration, with E kept
// implicit: for a block Z, E Z = W - Q C with W = A Z and C = Q^T W.  The
// host stores [Q | W] side by side (L + 16 columns), the Gram kernel forms
// its chunk partials, and this kernel reads C from the partial tiles (Q-block
// rows, W-block column), summed in chunk order, and writes the coefficient
// matrix M = [-C; I_b] ((L + 16) x 16, FP64), so that E Z = [Q | W] M is one
// FP64 apply.  Columns b..15 of M are zero.
__global__ __launch_bounds__(256) void proj_coef_kernel(const double* __restrict__ part, int nchunks, int L, int b,
                                                        double* __restrict__ M) {
    const int nt = L / 16 + 1, npairs = nt * (nt + 1) / 2, tw = nt - 1;
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < (L + 16) * 16; idx += 256 * gridDim.x) {
        const int a = idx >> 4, c = idx & 15;
        double v = 0.0;
        if (c < b) {
            if (a < L) {
                const int ta = a >> 4;
                const int pr = ta * nt - ta * (ta - 1) / 2 + (tw - ta);    // row-major upper-triangle index
                const int e = (a & 15) * 16 + c;
                double sum = 0.0;
                for (int ch = 0; ch < nchunks; ++ch) sum += part[((size_t)ch * npairs + pr) * 256 + e];
                v = -sum;
            } else {
                v = (a - L == c) ? 1.0 : 0.0;
            }
        }
        M[idx] = v;
    }
}

hipError_t launch_proj_coef(const double* partials, int64_t rows, int L, int b, double* M, hipStream_t s) {
    hipLaunchKernelGGL(proj_coef_kernel, dim3((unsigned)ceil_div((L + 16) * 16, 256)), dim3(256), 0, s, partials,
                       gram_chunks(rows), L, b, M);
    return hipGetLastError();
}

// residual[0] = largest Ritz value of the estimator; residual[1] = 0 when the
// Frobenius norm was not requested.
__global__ void residual_spec_final_kernel(const double* sigma, double* out, int fro_requested) {
    if (threadIdx.x == 0) {
        out[0] = sigma[0];
        if (!fro_requested) out[1] = 0.0;
    }
}

hipError_t launch_residual_spec_final(const double* sigma, double* out, int fro_requested, hipStream_t s) {
    hipLaunchKernelGGL(residual_spec_final_kernel, dim3(1), dim3(64), 0, s, sigma, out, fro_requested);
    return hipGetLastError();
}

}  // namespace rsvd
