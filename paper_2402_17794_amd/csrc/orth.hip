// Orthonormalisation (the "orth" of Algorithms 1-4) on gfx950.
//
// orth(Y) for a tall rows x l matrix Y is computed by CholeskyQR2:
//   G1 = Y^T Y, G1 = R1^T R1, Q1 = Y R1^{-1};  G2 = Q1^T Q1, G2 = R2^T R2,
//   Q = Q1 R2^{-1}.
// The Gram matrices, the Cholesky factors, their inverses and the products
// with the inverses are all computed in FP64, whatever the storage type of
// Y (FP32 products are exact in FP64), so one pass already orthonormalises
// to about kappa(Y)^2 * 2^-53 and the second pass brings Q to the storage
// precision.  diag(R) > 0, so Q is the Q factor of the thin QR of Y, the
// same matrix a Householder QR with non-negative diagonal produces.
//
// A pivot that is not clearly positive (rank-deficient or numerically
// rank-deficient Y, zero Y, NaN) marks the orthonormalisation as failed in a
// device flag; the remaining CholeskyQR kernels then return at once and a
// single-workgroup Householder QR recomputes Q from Y.  The flag lives in
// device memory, so the host never synchronises to choose the path.
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "../../include/rsvd.h"

namespace rsvd {

// ---------------------------------------------------------------- Gram --
// G = Y^T Y in FP64.  Output tiles of 32 x 32 on and above the diagonal;
// rows split into chunks of kGramRows.  Each workgroup computes one tile
// over one chunk; the last chunk to finish a tile (device-scope counter)
// sums the chunk partials in chunk order, writes the tile and its mirror.
constexpr int kGramRows = 256;
constexpr int kGT = 32;

int gram_pairs(int L) {
    const int nt = (int)ceil_div(L, kGT);
    return nt * (nt + 1) / 2;
}
size_t gram_partials_elems(int64_t rows, int L) {
    return (size_t)ceil_div(std::max<int64_t>(rows, 1), kGramRows) * gram_pairs(L) * kGT * kGT;
}

template <typename T>
__global__ __launch_bounds__(256) void gram_kernel(const T* __restrict__ Y, int64_t ldy, int64_t rows, int L,
                                                   double* __restrict__ G, double* __restrict__ part,
                                                   int* __restrict__ cnt, const DevFlags* skip) {
    if (skip && skip->orth_fail) return;
    const int nt = (int)ceil_div(L, kGT);
    const int npairs = nt * (nt + 1) / 2;
    const int pair = blockIdx.x % npairs;
    const int chunk = blockIdx.x / npairs;
    const int nchunks = (int)ceil_div(max<int64_t>(rows, 1), kGramRows);
    int a = 0, p = pair;
    while (p >= nt - a) { p -= nt - a; ++a; }
    const int b = a + p;

    __shared__ double Ya[kGT][kGT + 1];
    __shared__ double Yb[kGT][kGT + 1];
    const int tid = threadIdx.x;
    const int ti = (tid >> 4) * 2, tj = (tid & 15) * 2;
    double s00 = 0, s01 = 0, s10 = 0, s11 = 0;
    const int64_t r0 = (int64_t)chunk * kGramRows;
    const int64_t r1 = min<int64_t>(rows, r0 + kGramRows);
    for (int64_t rb = r0; rb < r1; rb += kGT) {
        __syncthreads();
        for (int idx = tid; idx < kGT * kGT; idx += 256) {
            const int rr = idx / kGT, cc = idx % kGT;
            const int64_t row = rb + rr;
            const int ca = a * kGT + cc, cb = b * kGT + cc;
            Ya[rr][cc] = (row < r1 && ca < L) ? (double)Y[row * ldy + ca] : 0.0;
            Yb[rr][cc] = (row < r1 && cb < L) ? (double)Y[row * ldy + cb] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int rr = 0; rr < kGT; ++rr) {
            const double x0 = Ya[rr][ti], x1 = Ya[rr][ti + 1];
            const double y0 = Yb[rr][tj], y1 = Yb[rr][tj + 1];
            s00 = fma(x0, y0, s00); s01 = fma(x0, y1, s01);
            s10 = fma(x1, y0, s10); s11 = fma(x1, y1, s11);
        }
    }
    double* mine = part + ((size_t)chunk * npairs + pair) * (kGT * kGT);
    mine[ti * kGT + tj] = s00;       mine[ti * kGT + tj + 1] = s01;
    mine[(ti + 1) * kGT + tj] = s10; mine[(ti + 1) * kGT + tj + 1] = s11;
    __threadfence();
    __syncthreads();
    __shared__ int last;
    if (tid == 0) last = (atomicAdd(&cnt[pair], 1) == nchunks - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int idx = tid; idx < kGT * kGT; idx += 256) {
        double s = 0.0;
        for (int c = 0; c < nchunks; ++c) s += part[((size_t)c * npairs + pair) * (kGT * kGT) + idx];
        const int i = a * kGT + idx / kGT, j = b * kGT + idx % kGT;
        if (i < L && j < L) {
            G[(int64_t)i * L + j] = s;
            G[(int64_t)j * L + i] = s;
        }
    }
    if (tid == 0) cnt[pair] = 0;
}

hipError_t launch_gram(int dtype, const void* Y, int64_t ldy, int64_t rows, int L, double* G, double* partials,
                       int* counters, const DevFlags* skip, hipStream_t s) {
    const int nchunks = (int)ceil_div(std::max<int64_t>(rows, 1), kGramRows);
    dim3 grid(nchunks * gram_pairs(L));
    if (dtype == 0)
        hipLaunchKernelGGL(gram_kernel<double>, grid, dim3(256), 0, s, (const double*)Y, ldy, rows, L, G, partials,
                           counters, skip);
    else
        hipLaunchKernelGGL(gram_kernel<float>, grid, dim3(256), 0, s, (const float*)Y, ldy, rows, L, G, partials,
                           counters, skip);
    return hipGetLastError();
}

// ------------------------------------------------------------ Cholesky --
// One workgroup factors the leading l x l block of G = R^T R and forms
// R^{-1} in the same sweep: row operations of the elimination are applied to
// an identity carried in the (otherwise unused) strict lower triangle, which
// turns into R^{-T} (the Gauss-Jordan view of Cholesky).  One barrier per
// column.  Row j of R and column j of R^{-1} are written as soon as pivot j
// is known.
constexpr int kCholLdsMax = 128;

template <bool IN_LDS>
__global__ __launch_bounds__(1024) void chol_kernel(const double* __restrict__ G, int l, int L,
                                                    double* __restrict__ R, double* __restrict__ Rinv,
                                                    DevFlags* flags, int mode, double* shift_out,
                                                    double* __restrict__ work) {
    __shared__ double lds[IN_LDS ? kCholLdsMax * kCholLdsMax : 1];
    if (mode == 1 && flags->orth_fail) return;
    double* M = IN_LDS ? lds : work;
    const int tid = threadIdx.x, nth = blockDim.x;

    double gmax = 0.0;
    bool nonfinite = false;
    for (int j = 0; j < l; ++j) {
        const double d = G[(int64_t)j * L + j];
        if (!isfinite(d)) nonfinite = true;
        else gmax = fmax(gmax, d);
    }
    const double rel = (mode == 0) ? 1e-12 : (mode == 1 ? 1e-2 : 0.0);
    double shift = 0.0;
    bool broke = false;
    for (int attempt = 0; attempt < (mode == 2 ? 5 : 1); ++attempt) {
        __syncthreads();
        for (int idx = tid; idx < L * L; idx += nth) { R[idx] = 0.0; Rinv[idx] = 0.0; }
        for (int idx = tid; idx < l * l; idx += nth) {
            const int a = idx / l, c = idx % l;
            M[idx] = (c >= a) ? G[(int64_t)a * L + c] + (a == c ? shift : 0.0) : 0.0;
        }
        __syncthreads();
        broke = nonfinite;
        for (int j = 0; j < l && !broke; ++j) {
            const double d = M[j * l + j];
            const double dj0 = G[(int64_t)j * L + j] + shift;
            if (!(d > rel * dj0) || !(d > 0.0) || !isfinite(d)) { broke = true; break; }
            const double rj = sqrt(d), inv_rj = 1.0 / rj, inv_d = 1.0 / d;
            for (int c = tid; c < l; c += nth) {
                if (c >= j) R[(int64_t)j * L + c] = M[j * l + c] * inv_rj;
                if (c < j) Rinv[(int64_t)c * L + j] = M[j * l + c] * inv_rj;
                if (c == j) Rinv[(int64_t)j * L + j] = inv_rj;
            }
            const int nrows = l - 1 - j;
            for (int idx = tid; idx < nrows * l; idx += nth) {
                const int a = j + 1 + idx / l, c = idx % l;
                const double f = M[j * l + a] * inv_d;
                if (c >= a || c < j) M[a * l + c] -= f * M[j * l + c];
                else if (c == j) M[a * l + j] = -f;
            }
            __syncthreads();
        }
        if (!broke || mode != 2 || nonfinite) break;
        shift = (shift == 0.0) ? gmax * 0x1.0p-40 : shift * 1024.0;
        if (!(shift > 0.0)) shift = 0x1.0p-1000;
    }
    if (tid == 0) {
        if (mode == 2) {
            *shift_out = shift;
            if (shift > 0.0) atomicOr(&flags->info, RSVD_INFO_SHIFTED_CHOLESKY);
            if (broke) atomicOr(&flags->info, RSVD_INFO_NONFINITE);
        } else {
            flags->orth_fail = broke ? 1 : 0;
        }
        if (nonfinite) atomicOr(&flags->info, RSVD_INFO_NONFINITE);
    }
}

hipError_t launch_chol(const double* G, int l, int L, double* R, double* Rinv, DevFlags* flags, int mode,
                       double* shift_out, double* work, hipStream_t s) {
    if (l <= kCholLdsMax)
        hipLaunchKernelGGL(chol_kernel<true>, dim3(1), dim3(1024), 0, s, G, l, L, R, Rinv, flags, mode, shift_out,
                           work);
    else
        hipLaunchKernelGGL(chol_kernel<false>, dim3(1), dim3(1024), 0, s, G, l, L, R, Rinv, flags, mode, shift_out,
                           work);
    return hipGetLastError();
}

// --------------------------------------------------------------- apply --
// out = in * M with FP64 accumulation: the CholeskyQR products Y R^{-1}, and
// the lifts U = Q U~ and V = B^T U~ Sigma^{-1}.  A workgroup owns 32 rows;
// thread (rg, cg) owns rows 2rg, 2rg+1 and output columns cg + 16c.  Inner
// dimension staged through LDS 16 at a time.
constexpr int kApplyRows = 32;
int apply_blocks(int64_t rows) { return (int)ceil_div(rows, kApplyRows); }

template <typename T, int CT>
__global__ __launch_bounds__(256) void apply_kernel(const T* __restrict__ in, int64_t ldi, int64_t rows, int L,
                                                    const double* __restrict__ M, int ldm, int ncols_out,
                                                    T* __restrict__ out, int64_t ldo, int transpose_out,
                                                    const double* __restrict__ colscale, const DevFlags* skip,
                                                    double* __restrict__ amax_val, int* __restrict__ amax_idx) {
    if (skip && skip->orth_fail) return;
    __shared__ double inS[kApplyRows][17];
    __shared__ double MS[16][CT * 16 + 1];
    const int tid = threadIdx.x, rg = tid >> 4, cg = tid & 15;
    const int64_t row0 = (int64_t)blockIdx.x * kApplyRows;
    double acc0[CT], acc1[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) { acc0[c] = 0.0; acc1[c] = 0.0; }
    for (int a0 = 0; a0 < L; a0 += 16) {
        __syncthreads();
        for (int idx = tid; idx < kApplyRows * 16; idx += 256) {
            const int rr = idx >> 4, aa = idx & 15;
            const int64_t row = row0 + rr;
            inS[rr][aa] = (row < rows && a0 + aa < L) ? (double)in[row * ldi + a0 + aa] : 0.0;
        }
        for (int idx = tid; idx < 16 * CT * 16; idx += 256) {
            const int aa = idx / (CT * 16), cc = idx % (CT * 16);
            MS[aa][cc] = (a0 + aa < L && cc < ncols_out) ? M[(int64_t)(a0 + aa) * ldm + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int aa = 0; aa < 16; ++aa) {
            const double x0 = inS[2 * rg][aa], x1 = inS[2 * rg + 1][aa];
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const double mv = MS[aa][cg + 16 * c];
                acc0[c] = fma(x0, mv, acc0[c]);
                acc1[c] = fma(x1, mv, acc1[c]);
            }
        }
    }
    extern __shared__ double av_dyn[];          // kApplyRows x (CT * 16 + 1), argmax only
    auto av = [&](int rr, int col) -> double& { return av_dyn[rr * (CT * 16 + 1) + col]; };
    const int64_t ra = row0 + 2 * rg, rb = ra + 1;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int col = cg + 16 * c;
        if (col >= ncols_out) continue;
        const double sc = colscale ? colscale[col] : 1.0;
        const T v0 = (T)(acc0[c] * sc), v1 = (T)(acc1[c] * sc);
        if (!transpose_out) {
            if (ra < rows) out[ra * ldo + col] = v0;
            if (rb < rows) out[rb * ldo + col] = v1;
        } else {
            if (ra < rows) out[(int64_t)col * ldo + ra] = v0;
            if (rb < rows) out[(int64_t)col * ldo + rb] = v1;
        }
        if (amax_val) {
            av(2 * rg, col) = (ra < rows) ? (double)v0 : 0.0;
            av(2 * rg + 1, col) = (rb < rows) ? (double)v1 : 0.0;
        }
    }
    if (!amax_val) return;
    __syncthreads();
    for (int col = tid; col < ncols_out; col += 256) {
        double best = -1.0, val = 0.0;
        int bi = 0;
        for (int rr = 0; rr < kApplyRows; ++rr)      // lowest row wins ties
            if (fabs(av(rr, col)) > best) { best = fabs(av(rr, col)); val = av(rr, col); bi = rr; }
        amax_val[(int64_t)blockIdx.x * ncols_out + col] = val;
        amax_idx[(int64_t)blockIdx.x * ncols_out + col] = (int)(row0 + bi);
    }
}

template <typename T>
static hipError_t apply_dispatch(int CT, dim3 grid, hipStream_t s, const T* in, int64_t ldi, int64_t rows, int L,
                                 const double* M, int ldm, int ncols_out, T* out, int64_t ldo, int tr,
                                 const double* colscale, const DevFlags* skip, double* av, int* ai) {
#define RSVD_CT_CASE(N)                                                                                         \
    case N:                                                                                                     \
        hipLaunchKernelGGL((apply_kernel<T, N>), grid, dim3(256),                                               \
                           av ? (size_t)kApplyRows * (N * 16 + 1) * sizeof(double) : 0, s, in, ldi, rows, L, M,  \
                           ldm, ncols_out, out, ldo, tr, colscale, skip, av, ai);                               \
        break;
    switch (CT) {
        RSVD_CT_CASE(1) RSVD_CT_CASE(2) RSVD_CT_CASE(3) RSVD_CT_CASE(4) RSVD_CT_CASE(5) RSVD_CT_CASE(6)
        RSVD_CT_CASE(7) RSVD_CT_CASE(8) RSVD_CT_CASE(9) RSVD_CT_CASE(10) RSVD_CT_CASE(11) RSVD_CT_CASE(12)
        RSVD_CT_CASE(13) RSVD_CT_CASE(14) RSVD_CT_CASE(15) RSVD_CT_CASE(16) RSVD_CT_CASE(17) RSVD_CT_CASE(18)
        default: return hipErrorInvalidValue;
    }
#undef RSVD_CT_CASE
    return hipGetLastError();
}

hipError_t launch_apply(int dtype, const void* in, int64_t ldi, int64_t rows, int L, const double* M, int ldm,
                        int ncols_out, void* out, int64_t ldo, int transpose_out, const double* colscale,
                        const DevFlags* skip, double* av, int* ai, hipStream_t s) {
    if (rows == 0 || ncols_out == 0) return hipSuccess;
    const int CT = (int)ceil_div(ncols_out, 16);
    dim3 grid(apply_blocks(rows));
    if (dtype == 0)
        return apply_dispatch<double>(CT, grid, s, (const double*)in, ldi, rows, L, M, ldm, ncols_out, (double*)out,
                                      ldo, transpose_out, colscale, skip, av, ai);
    return apply_dispatch<float>(CT, grid, s, (const float*)in, ldi, rows, L, M, ldm, ncols_out, (float*)out, ldo,
                                 transpose_out, colscale, skip, av, ai);
}

// ---------------------------------------------------------- Householder --
// Fallback thin QR by Householder reflections in one workgroup of 16
// wavefronts, working in FP64 in device scratch (H: reflectors / R,
// Qw: the explicit Q).  Column j: reflect the trailing part onto
// -sign(x_0) |x| e_1 and apply the reflector to the trailing columns
// (wavefront c handles columns c, c + 16, ...).  Q is formed by applying the
// reflectors last to first to the first l columns of the identity; columns
// whose diagonal of R is negative are negated so that diag(R) >= 0.
template <typename T>
__global__ __launch_bounds__(1024) void householder_kernel(const T* __restrict__ Y, int64_t ldy, int64_t rows, int l,
                                                           int L, T* __restrict__ Q, int64_t ldq,
                                                           double* __restrict__ H, double* __restrict__ Qw,
                                                           DevFlags* flags, int force, int pad_cols) {
    if (!force && !flags->orth_fail) return;
    __shared__ double tau[kMaxL], beta[kMaxL], red[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t idx = tid; idx < rows * L; idx += 1024) {
        const int64_t i = idx / L;
        const int c = (int)(idx % L);
        H[idx] = c < l ? (double)Y[i * ldy + c] : 0.0;
        Qw[idx] = (c < l && i == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < l; ++j) {
        double s = 0.0;
        for (int64_t i = j + tid; i < rows; i += 1024) s += H[i * L + j] * H[i * L + j];
        s = block_sum(s, red);
        const double alpha = H[(int64_t)j * L + j];
        const double normx = sqrt(s);
        __syncthreads();
        if (normx == 0.0) {
            if (tid == 0) { tau[j] = 0.0; beta[j] = 0.0; }
            continue;
        }
        const double bj = alpha >= 0.0 ? -normx : normx;
        const double v0 = alpha - bj;
        const double vtv = s - alpha * alpha + v0 * v0;
        const double tj = 2.0 / vtv;
        if (tid == 0) { H[(int64_t)j * L + j] = v0; tau[j] = tj; beta[j] = bj; }
        __syncthreads();
        for (int c = j + 1 + wave; c < l; c += 16) {
            double w = 0.0;
            for (int64_t i = j + lane; i < rows; i += 64) w += H[i * L + j] * H[i * L + c];
            w = wave_sum(w) * tj;
            for (int64_t i = j + lane; i < rows; i += 64) H[i * L + c] -= w * H[i * L + j];
        }
        __syncthreads();
    }
    for (int j = l - 1; j >= 0; --j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;
        for (int c = j + wave; c < l; c += 16) {
            double w = 0.0;
            for (int64_t i = j + lane; i < rows; i += 64) w += H[i * L + j] * Qw[i * L + c];
            w = wave_sum(w) * tj;
            for (int64_t i = j + lane; i < rows; i += 64) Qw[i * L + c] -= w * H[i * L + j];
        }
        __syncthreads();
    }
    for (int64_t idx = tid; idx < rows * L; idx += 1024) {
        const int64_t i = idx / L;
        const int c = (int)(idx % L);
        if (c < l) Q[i * ldq + c] = (T)(beta[c] < 0.0 ? -Qw[idx] : Qw[idx]);
        else if (c < pad_cols) Q[i * ldq + c] = (T)0;
    }
    if (tid == 0) atomicOr(&flags->info, RSVD_INFO_QR_FALLBACK);
}

hipError_t launch_householder(int dtype, const void* Y, int64_t ldy, int64_t rows, int l, int L, void* Q,
                              int64_t ldq, double* H, double* Qw, DevFlags* flags, int force, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL(householder_kernel<double>, dim3(1), dim3(1024), 0, s, (const double*)Y, ldy, rows, l, L,
                           (double*)Q, ldq, H, Qw, flags, force, L);
    else
        hipLaunchKernelGGL(householder_kernel<float>, dim3(1), dim3(1024), 0, s, (const float*)Y, ldy, rows, l, L,
                           (float*)Q, ldq, H, Qw, flags, force, L);
    return hipGetLastError();
}

}  // namespace rsvd
