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

// Round-robin (circle method) schedule: with n2 (even) columns, round r pairs
// slot 0 with (n2 - 1, r) and slot s > 0 with ((r + s), (r - s)) mod (n2 - 1).
__device__ __forceinline__ void rr_pair(int r, int s, int n2, int& p1, int& p2) {
    const int m = n2 - 1;
    if (s == 0) { p1 = m; p2 = r; }
    else { p1 = (r + s) % m; p2 = (r - s + m) % m; }
}

template <int RPL, bool IN_LDS>
__global__ __launch_bounds__(1024) void jacobi_kernel(const double* __restrict__ R, int l, int L,
                                                      const double* __restrict__ shift_p, double* __restrict__ sigma,
                                                      double* __restrict__ Ut, double* __restrict__ Mv,
                                                      DevFlags* flags, double* __restrict__ work) {
    __shared__ double lds[IN_LDS ? kJacobiLdsMax * kJacobiLdsMax : 1];
    __shared__ int rotated;
    __shared__ double nrm2[kMaxL];
    __shared__ int rank_of[kMaxL];
    double* X = IN_LDS ? lds : work;           // column-major, X[c * l + r] = R[c][r]
    const int tid = threadIdx.x, q = tid >> 4, e = tid & 15;

    for (int idx = tid; idx < l * l; idx += 1024) {
        const int c = idx / l, r = idx % l;
        X[idx] = R[(int64_t)c * L + r];
    }
    const int n2 = l + (l & 1);
    bool converged = (l < 2);
    __syncthreads();
    for (int sweep = 0; sweep < kJacobiMaxSweeps && !converged; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < n2 - 1; ++r) {
            for (int s = q; s < n2 / 2; s += 64) {
                int p1, p2;
                rr_pair(r, s, n2, p1, p2);
                if (p1 >= l || p2 >= l) continue;
                const int i = min(p1, p2), j = max(p1, p2);
                double xi[RPL], xj[RPL];
                double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
                for (int t = 0; t < RPL; ++t) {
                    const int row = e + 16 * t;
                    xi[t] = row < l ? X[i * l + row] : 0.0;
                    xj[t] = row < l ? X[j * l + row] : 0.0;
                    a = fma(xi[t], xi[t], a);
                    b = fma(xj[t], xj[t], b);
                    g = fma(xi[t], xj[t], g);
                }
                a = quarter_sum(a);
                b = quarter_sum(b);
                g = quarter_sum(g);
                if (fabs(g) > kJacobiTol * sqrt(a * b)) {
                    const double zeta = (b - a) / (2.0 * g);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll
                    for (int u = 0; u < RPL; ++u) {
                        const int row = e + 16 * u;
                        if (row < l) {
                            X[i * l + row] = c * xi[u] - sn * xj[u];
                            X[j * l + row] = sn * xi[u] + c * xj[u];
                        }
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

    for (int c = q; c < l; c += 64) {
        double s2 = 0.0;
        for (int row = e; row < l; row += 16) s2 = fma(X[c * l + row], X[c * l + row], s2);
        s2 = quarter_sum(s2);
        if (e == 0) nrm2[c] = s2;
    }
    __syncthreads();
    const double shift = *shift_p;
    // Stable descending order of the singular values sqrt(max(nrm2 - shift, 0)).
    for (int c = tid; c < l; c += 1024) {
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
    for (int idx = tid; idx < L * L; idx += 1024) {
        Ut[idx] = 0.0;
        Mv[idx] = 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < l * l; idx += 1024) {
        const int c = idx / l, row = idx % l;
        const double nc = sqrt(nrm2[c]);
        const double sc = sqrt(fmax(nrm2[c] - shift, 0.0));
        const double u = nc > 0.0 ? X[c * l + row] / nc : (row == c ? 1.0 : 0.0);
        const int col = rank_of[c];
        Ut[(int64_t)row * L + col] = u;
        Mv[(int64_t)row * L + col] = sc > 0.0 ? u / sc : 0.0;
    }
}

hipError_t launch_jacobi(const double* R, int l, int L, const double* shift, double* sigma, double* Ut, double* Mv,
                         DevFlags* flags, double* work, hipStream_t s) {
    if (l <= kJacobiLdsMax)
        hipLaunchKernelGGL((jacobi_kernel<kJacobiLdsMax / 16, true>), dim3(1), dim3(1024), 0, s, R, l, L, shift, sigma,
                           Ut, Mv, flags, work);
    else
        hipLaunchKernelGGL((jacobi_kernel<kMaxL / 16, false>), dim3(1), dim3(1024), 0, s, R, l, L, shift, sigma, Ut,
                           Mv, flags, work);
    return hipGetLastError();
}

// Signs: for each returned column c of V, the entry of largest magnitude
// (lowest row on ties) is made positive.  Block partials arrive in row order.
__global__ void signs_kernel(const double* __restrict__ av, const int* __restrict__ ai, int nblocks, int r,
                             const double* __restrict__ sigma, double* __restrict__ S_out, double* __restrict__ sign) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < r; c += gridDim.x * blockDim.x) {
        double best = -1.0, val = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            const double v = av[(int64_t)b * r + c];
            if (fabs(v) > best) { best = fabs(v); val = v; }
        }
        (void)ai;
        sign[c] = val < 0.0 ? -1.0 : 1.0;
        S_out[c] = sigma[c];
    }
}

hipError_t launch_signs(const double* av, const int* ai, int nblocks, int r, const double* sigma, double* S_out,
                        double* sign, hipStream_t s) {
    hipLaunchKernelGGL(signs_kernel, dim3((unsigned)ceil_div(r, 256)), dim3(256), 0, s, av, ai, nblocks, r, sigma,
                       S_out, sign);
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
// stored Q and B^T, sums its squares, and the last workgroup (device-scope
// counter) adds the tile sums in tile order.
constexpr int kResTile = 64;

size_t residual_partials(int64_t m, int64_t n) {
    return (size_t)ceil_div(m, kResTile) * (size_t)ceil_div(n, kResTile);
}

template <typename T>
__global__ __launch_bounds__(256) void residual_fro_kernel(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                           const T* __restrict__ Q, const T* __restrict__ Bt, int L,
                                                           double* __restrict__ part, int* __restrict__ cnt,
                                                           double* __restrict__ out) {
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
    __threadfence();
    __syncthreads();
    __shared__ int last;
    if (tid == 0) last = (atomicAdd(cnt, 1) == (int)gridDim.x - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (tid == 0) {
        double t = 0.0;
        for (unsigned b = 0; b < gridDim.x; ++b) t += part[b];
        out[0] = 0.0;
        out[1] = sqrt(t);
        *cnt = 0;
    }
}

hipError_t launch_residual_fro(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, const void* Q,
                               const void* Bt, int l, int L, double* partial, int* counter, double* out,
                               hipStream_t s) {
    (void)l;
    dim3 grid((unsigned)residual_partials(m, n));
    if (dtype == 0)
        hipLaunchKernelGGL(residual_fro_kernel<double>, grid, dim3(256), 0, s, (const double*)A, lda, m, n,
                           (const double*)Q, (const double*)Bt, L, partial, counter, out);
    else
        hipLaunchKernelGGL(residual_fro_kernel<float>, grid, dim3(256), 0, s, (const float*)A, lda, m, n,
                           (const float*)Q, (const float*)Bt, L, partial, counter, out);
    return hipGetLastError();
}

}  // namespace rsvd
