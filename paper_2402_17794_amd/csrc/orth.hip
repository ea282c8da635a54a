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
// Partial Gram matrices Y_c^T Y_c (FP64, on FP64 MFMA 16x16x4) for nchunks
// row chunks Y_c of Y.  Output tiles of 16 x 16 on and above the diagonal.
// A workgroup of 4 wavefronts computes one tile over one chunk: wavefront w
// takes the 4-row steps w, w + 4, ... with two accumulators, and the eight
// accumulators are summed in a fixed order.  The chunk partials are summed
// (in chunk order) by the Cholesky kernel that consumes them, so no
// workgroup ever waits for another.
int gram_pairs(int L) {
    const int nt = (int)ceil_div(L, 16);
    return nt * (nt + 1) / 2;
}
int gram_chunks(int64_t rows) { return (int)std::min<int64_t>(8, std::max<int64_t>(1, ceil_div(rows, 1024))); }
size_t gram_partials_elems(int64_t rows, int L) { return (size_t)gram_chunks(rows) * gram_pairs(L) * 256; }

template <typename T>
__global__ __launch_bounds__(256) void gram_kernel(const T* __restrict__ Y, int64_t ldy, int64_t rows, int L,
                                                   int nchunks, double* __restrict__ part, const DevFlags* skip) {
    if (skip && skip->orth_fail) return;
    const int nt = L / 16;
    const int npairs = nt * (nt + 1) / 2;
    const int pair = blockIdx.x % npairs;
    const int chunk = blockIdx.x / npairs;
    int a = 0, p = pair;
    while (p >= nt - a) { p -= nt - a; ++a; }
    const int b = a + p;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t per = round_up(ceil_div(rows, nchunks), 16);
    const int64_t r0 = (int64_t)chunk * per;
    const int64_t r1 = min<int64_t>(rows, r0 + per);
    const T* __restrict__ ya = Y + a * 16 + li;
    const T* __restrict__ yb = Y + b * 16 + li;
    doublex4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    constexpr int UNR = 8;          // 8 MFMA steps (32 rows per wavefront) per batch of loads
    for (int64_t k0 = r0 + 4 * wave; k0 < r1; k0 += 16 * UNR) {
        double va[UNR], vb[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t row = k0 + 16 * u + lk;
            const bool ok = row < r1;
            va[u] = ok ? (double)ya[row * ldy] : 0.0;
            vb[u] = ok ? (double)yb[row * ldy] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UNR; u += 2) {
            acc0 = mfma16x16x4(va[u], vb[u], acc0);
            acc1 = mfma16x16x4(va[u + 1], vb[u + 1], acc1);
        }
    }
    // acc[v] = G[a*16 + acc_row(lk, v)][b*16 + li] restricted to this chunk.
    __shared__ double red[4][256];
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][acc_row<double>(lk, v) * 16 + li] = acc0[v] + acc1[v];
    __syncthreads();
    part[((size_t)chunk * npairs + pair) * 256 + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

hipError_t launch_gram(int dtype, const void* Y, int64_t ldy, int64_t rows, int L, double* partials,
                       const DevFlags* skip, hipStream_t s) {
    const int nchunks = gram_chunks(rows);
    dim3 grid(nchunks * gram_pairs(L));
    if (dtype == 0)
        hipLaunchKernelGGL(gram_kernel<double>, grid, dim3(256), 0, s, (const double*)Y, ldy, rows, L, nchunks,
                           partials, skip);
    else
        hipLaunchKernelGGL(gram_kernel<float>, grid, dim3(256), 0, s, (const float*)Y, ldy, rows, L, nchunks,
                           partials, skip);
    return hipGetLastError();
}

// ------------------------------------------------------------ Cholesky --
// One workgroup factors the leading l x l block of G = R^T R and forms
// R^{-1} in the same sweep: row operations of the elimination are applied to
// an identity carried in the (otherwise unused) strict lower triangle, which
// turns into R^{-T} (the Gauss-Jordan view of Cholesky).  One barrier per
// column.  Thread (rg, cl) owns rows j+1+rg+32u and columns cl+32v of the
// trailing update; all its loads are issued before its updates.  Row j of R
// and column j of R^{-1} are written as soon as pivot j is known.
//
// Second pass of CholeskyQR2 (mode 1): G = Q1^T Q1 = I + E with E tiny.  If
// max |E| <= tau (FP32 data: 2^-13, FP64: 2^-26) the factor is taken to first
// order, R = I + U with U = triu(E) - diag(E) / 2 and R^{-1} = I - U; the
// neglected terms are O(|E|^2), below the storage precision, and Q1 R^{-1}
// is orthonormal to O(|E|^2).  Otherwise the exact factorisation runs.
constexpr int kCholLdsMax = 128;

template <bool IN_LDS>
__global__ __launch_bounds__(1024) void chol_kernel(const double* __restrict__ part, int nchunks, int l, int L,
                                                    double* __restrict__ R, double* __restrict__ Rinv,
                                                    DevFlags* flags, int mode, double* shift_out,
                                                    double* __restrict__ work, double tau) {
    constexpr int LP = IN_LDS ? kCholLdsMax : 1;
    __shared__ double lds[IN_LDS ? kCholLdsMax * kCholLdsMax : 1];
    __shared__ double dg[kMaxL];
    __shared__ double inv_r[kMaxL];
    __shared__ unsigned long long s_emax;
    if (mode == 1 && flags->orth_fail) return;
    double* M = IN_LDS ? lds : work;
    const int ldm = IN_LDS ? LP : l;
    const int tid = threadIdx.x, rg = tid >> 5, cl = tid & 31;
    const int nt = L / 16, npairs = nt * (nt + 1) / 2;

    // Sum the chunk partials (chunk order) into the upper triangle of M;
    // the strict lower triangle starts at zero.
    if (tid == 0) s_emax = 0ull;
    for (int a = rg; a < l; a += 32)
        for (int c = cl; c < a; c += 32) M[a * ldm + c] = 0.0;
    double emax = 0.0;
    for (int idx = tid; idx < npairs * 256; idx += 1024) {
        const int pr = idx >> 8, e = idx & 255;
        int ta = 0, pp = pr;
        while (pp >= nt - ta) { pp -= nt - ta; ++ta; }
        const int row = ta * 16 + (e >> 4), col = (ta + pp) * 16 + (e & 15);
        if (row > col || row >= l || col >= l) continue;
        double sum = 0.0;
        int c = 0;
        for (; c + 4 <= nchunks; c += 4) {
            const double x0 = part[((size_t)(c + 0) * npairs + pr) * 256 + e];
            const double x1 = part[((size_t)(c + 1) * npairs + pr) * 256 + e];
            const double x2 = part[((size_t)(c + 2) * npairs + pr) * 256 + e];
            const double x3 = part[((size_t)(c + 3) * npairs + pr) * 256 + e];
            sum = (((sum + x0) + x1) + x2) + x3;
        }
        for (; c < nchunks; ++c) sum += part[((size_t)c * npairs + pr) * 256 + e];
        M[row * ldm + col] = sum;
        if (row == col) dg[row] = sum;
        double ee = fabs(sum - (row == col ? 1.0 : 0.0));
        if (!(ee < 1e300)) ee = 1e300;
        emax = fmax(emax, ee);
    }
    if (mode == 1) atomicMax(&s_emax, (unsigned long long)__double_as_longlong(emax));
    __syncthreads();

    if (mode == 1 && __longlong_as_double((long long)s_emax) <= tau) {
        // Second pass: first-order factor (see above).
#pragma unroll 4
        for (int idx = tid; idx < L * L; idx += 1024) {
            const int a = idx / L, c = idx - a * L;
            double r = 0.0, ri = 0.0;
            if (a <= c && c < l) {
                const double e = M[a * ldm + c] - (a == c ? 1.0 : 0.0);
                const double u = a < c ? e : 0.5 * e;
                r = (a == c ? 1.0 : 0.0) + u;
                ri = (a == c ? 1.0 : 0.0) - u;
            }
            R[idx] = r;
            Rinv[idx] = ri;
        }
        if (tid == 0) flags->orth_fail = 0;
        return;
    }

    double gmax = 0.0;
    bool nonfinite = false;
    for (int j = 0; j < l; ++j) {
        const double d = dg[j];
        if (!isfinite(d)) nonfinite = true;
        else gmax = fmax(gmax, d);
    }
    const double rel = (mode == 0) ? 1e-12 : (mode == 1 ? 1e-2 : 0.0);
    double shift = 0.0, applied = 0.0;
    bool broke = false;
    for (int attempt = 0; attempt < (mode == 2 ? 5 : 1); ++attempt) {
        if (shift != applied) {        // retry: the factorisation overwrote M; restore with the new shift
            __syncthreads();
            for (int idx = tid; idx < npairs * 256; idx += 1024) {
                const int pr = idx >> 8, e = idx & 255;
                int ta = 0, pp = pr;
                while (pp >= nt - ta) { pp -= nt - ta; ++ta; }
                const int row = ta * 16 + (e >> 4), col = (ta + pp) * 16 + (e & 15);
                if (row > col || row >= l || col >= l) continue;
                double sum = 0.0;
                for (int c = 0; c < nchunks; ++c) sum += part[((size_t)c * npairs + pr) * 256 + e];
                M[row * ldm + col] = sum + (row == col ? shift : 0.0);
            }
            for (int a = rg; a < l; a += 32)
                for (int c = cl; c < a; c += 32) M[a * ldm + c] = 0.0;
            applied = shift;
            __syncthreads();
        }
        broke = nonfinite;
        for (int j = 0; j < l && !broke; ++j) {
            const double d = M[j * ldm + j];
            if (!(d > rel * (dg[j] + shift)) || !(d > 0.0) || !isfinite(d)) { broke = true; break; }
            const double inv_rj = 1.0 / sqrt(d), inv_d = inv_rj * inv_rj;
            if (tid == 0) inv_r[j] = inv_rj;
            if (IN_LDS) {
                // Rows a = j+1+rg+32u (u < 4), columns c = cl+32v (v < 4); l <= 128.
                double rowj[4], f[4], x[4][4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = cl + 32 * v;
                    rowj[v] = c < l ? M[j * ldm + c] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int a = min(j + 1 + rg + 32 * u, LP - 1);
                    f[u] = M[j * ldm + a] * inv_d;
#pragma unroll
                    for (int v = 0; v < 4; ++v) x[u][v] = M[a * ldm + cl + 32 * v];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int a = j + 1 + rg + 32 * u;
                    if (a >= l) continue;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int c = cl + 32 * v;
                        if (c >= l) continue;
                        if (c >= a || c < j) M[a * ldm + c] = x[u][v] - f[u] * rowj[v];
                        else if (c == j) M[a * ldm + j] = -f[u];
                    }
                }
            } else {
                for (int a = j + 1 + rg; a < l; a += 32) {
                    const double fa = M[j * ldm + a] * inv_d;
                    for (int c = cl; c < l; c += 32) {
                        if (c >= a || c < j) M[a * ldm + c] -= fa * M[j * ldm + c];
                        else if (c == j) M[a * ldm + j] = -fa;
                    }
                }
            }
            __syncthreads();
        }
        if (!broke || mode != 2 || nonfinite) break;
        shift = (shift == 0.0) ? gmax * 0x1.0p-40 : shift * 1024.0;
        if (!(shift > 0.0)) shift = 0x1.0p-1000;
    }
    __syncthreads();
    // Row a of M holds row a of R (times r_aa) in its upper part and row a of
    // R^{-T} (times r_aa) in its strict lower part; neither changes after step a.
    if (!broke) {
#pragma unroll 4
        for (int idx = tid; idx < L * L; idx += 1024) {
            const int x = idx / L, y = idx - x * L;
            double r = 0.0, ri = 0.0;
            if (x < l && y < l) {
                if (y >= x) r = M[x * ldm + y] * inv_r[x];
                if (x <= y) ri = (x == y) ? inv_r[y] : M[y * ldm + x] * inv_r[y];
            }
            R[idx] = r;
            Rinv[idx] = ri;
        }
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

// Blocked form for l <= 128 (the matrix lives in LDS).  Blocks of 16:
// step J factors the diagonal block by one wavefront (Gauss-Jordan on
// [D | I] in registers, one LDS row broadcast per column, no workgroup
// barrier), then the whole workgroup forms the panel R_J,K = R_JJ^{-T} G_J,K,
// the block column J of R^{-1} (X_IJ = -(sum_{I <= K < J} X_IK R_KJ) R_JJ^{-1})
// and the trailing update G_KK' -= R_JK^T R_JK'.  Three barriers per block
// instead of one per column.  Storage in M (LDS): upper triangle = R, strict
// lower triangle = R^{-1} transposed (X[a][c] at M[c][a]), inv_r = 1 / r_aa;
// rows and columns past l are padded with the identity.
__global__ __launch_bounds__(1024) void chol_blocked_kernel(const double* __restrict__ part, int nchunks, int l,
                                                            int L, double* __restrict__ R, double* __restrict__ Rinv,
                                                            DevFlags* flags, int mode, double* shift_out, double tau) {
    constexpr int LP = kCholLdsMax;
    __shared__ double M[LP * LP];
    __shared__ double T[7 * 256];               // T_IJ = sum_K X_IK R_KJ, I < J
    __shared__ double inv_r[LP];
    __shared__ double dg[LP];
    __shared__ double rowp[32];
    __shared__ int s_broke;
    __shared__ unsigned long long s_emax;
    if (mode == 1 && flags->orth_fail) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nt = L / 16, npairs = nt * (nt + 1) / 2;
    const int nb = (l + 15) / 16, lp = 16 * nb;

    auto load = [&](double shift) {
        for (int idx = tid; idx < lp * lp; idx += 1024) {
            const int a = idx / lp, c = idx - a * lp;
            M[a * LP + c] = (a >= l && a == c) ? 1.0 : 0.0;
        }
        __syncthreads();
        double emax = 0.0;
        for (int idx = tid; idx < npairs * 256; idx += 1024) {
            const int pr = idx >> 8, e = idx & 255;
            int ta = 0, pp = pr;
            while (pp >= nt - ta) { pp -= nt - ta; ++ta; }
            const int row = ta * 16 + (e >> 4), col = (ta + pp) * 16 + (e & 15);
            if (row > col || row >= l || col >= l) continue;
            double sum = 0.0;
            int c = 0;
            for (; c + 4 <= nchunks; c += 4) {
                const double x0 = part[((size_t)(c + 0) * npairs + pr) * 256 + e];
                const double x1 = part[((size_t)(c + 1) * npairs + pr) * 256 + e];
                const double x2 = part[((size_t)(c + 2) * npairs + pr) * 256 + e];
                const double x3 = part[((size_t)(c + 3) * npairs + pr) * 256 + e];
                sum = (((sum + x0) + x1) + x2) + x3;
            }
            for (; c < nchunks; ++c) sum += part[((size_t)c * npairs + pr) * 256 + e];
            if (row == col) dg[row] = sum;
            M[row * LP + col] = sum + (row == col ? shift : 0.0);
            double ee = fabs(sum - (row == col ? 1.0 : 0.0));
            if (!(ee < 1e300)) ee = 1e300;
            emax = fmax(emax, ee);
        }
        for (int a = l + tid; a < lp; a += 1024) dg[a] = 1.0;
        return emax;
    };

    if (tid == 0) { s_emax = 0ull; s_broke = 0; }
    __syncthreads();
    const double emax_t = load(0.0);
    if (mode == 1) atomicMax(&s_emax, (unsigned long long)__double_as_longlong(emax_t));
    __syncthreads();
    if (mode == 1 && __longlong_as_double((long long)s_emax) <= tau) {
#pragma unroll 4
        for (int idx = tid; idx < L * L; idx += 1024) {
            const int a = idx / L, c = idx - a * L;
            double r = 0.0, ri = 0.0;
            if (a <= c && c < l) {
                const double e = M[a * LP + c] - (a == c ? 1.0 : 0.0);
                const double u = a < c ? e : 0.5 * e;
                r = (a == c ? 1.0 : 0.0) + u;
                ri = (a == c ? 1.0 : 0.0) - u;
            }
            R[idx] = r;
            Rinv[idx] = ri;
        }
        if (tid == 0) flags->orth_fail = 0;
        return;
    }
    bool nonfinite = false;
    double gmax = 0.0;
    for (int j = 0; j < l; ++j) {
        const double d = dg[j];
        if (!isfinite(d)) nonfinite = true;
        else gmax = fmax(gmax, d);
    }
    const double rel = (mode == 0) ? 1e-12 : (mode == 1 ? 1e-2 : 0.0);
    double shift = 0.0;
    bool broke = nonfinite;
    for (int attempt = 0; attempt < (mode == 2 ? 5 : 1) && !nonfinite; ++attempt) {
        if (attempt > 0) {
            load(shift);
            if (tid == 0) s_broke = 0;
            __syncthreads();
        }
        for (int J = 0; J < nb; ++J) {
            const int j0 = 16 * J;
            // (a) diagonal block by wavefront 0.
            if (wave == 0) {
                const int i = lane;
                double u[16], e[16];
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    u[c] = (i < 16 && c >= i) ? M[(j0 + i) * LP + j0 + c] : 0.0;
                    e[c] = (c == i) ? 1.0 : 0.0;
                }
                bool bad = false;
#pragma unroll
                for (int p = 0; p < 16; ++p) {
                    if (i == p) {
#pragma unroll
                        for (int c = 0; c < 16; ++c) { rowp[c] = u[c]; rowp[16 + c] = e[c]; }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    const double d = rowp[p];
                    if (!(d > rel * (dg[j0 + p] + shift)) || !(d > 0.0) || !isfinite(d)) bad = true;
                    if (i > p && i < 16) {
                        const double f = rowp[i] / d;
#pragma unroll
                        for (int c = 0; c < 16; ++c) {
                            if (c >= i) u[c] -= f * rowp[c];
                            if (c <= p) e[c] -= f * rowp[16 + c];
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
                if (i < 16) {
                    const double inv = 1.0 / sqrt(u[i]);
#pragma unroll
                    for (int c = 0; c < 16; ++c) {
                        if (c >= i) M[(j0 + i) * LP + j0 + c] = u[c] * inv;
                        else M[(j0 + i) * LP + j0 + c] = e[c] * inv;
                    }
                    inv_r[j0 + i] = inv;
                }
                if (bad && lane == 0) s_broke = 1;
            }
            __syncthreads();
            if (s_broke) break;
            // (b) panel R_J,K (one thread per column) and T_IJ = sum_{I<=K<J} X_IK R_KJ.
            {
                const int ncols = lp - j0 - 16;
                if (tid < ncols) {
                    const int c = j0 + 16 + tid;
                    double g[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) g[k] = M[(j0 + k) * LP + c];
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        double acc = g[i] * inv_r[j0 + i];
#pragma unroll
                        for (int k = 0; k < 16; ++k)
                            if (k < i) acc = fma(M[(j0 + i) * LP + j0 + k], g[k], acc);
                        M[(j0 + i) * LP + c] = acc;
                    }
                }
                for (int idx = tid - 128; idx >= 0 && idx < J * 256; idx += 1024 - 128) {
                    const int I = idx >> 8, i = (idx >> 4) & 15, c = idx & 15;
                    double acc = 0.0;
                    for (int K = I; K < J; ++K) {
#pragma unroll
                        for (int k = 0; k < 16; ++k) {
                            const int a = 16 * I + i, b = 16 * K + k;   // X[a][b], b >= a
                            const double x = (b == a) ? inv_r[a] : (b > a ? M[b * LP + a] : 0.0);
                            acc = fma(x, M[b * LP + j0 + c], acc);
                        }
                    }
                    T[(I * 16 + i) * 16 + c] = acc;
                }
            }
            __syncthreads();
            // (c) trailing update and X_IJ = -T_IJ R_JJ^{-1}.
            {
                const int t0 = j0 + 16, nt2 = lp - t0;
                for (int idx = tid; idx < nt2 * nt2; idx += 1024) {
                    const int r = t0 + idx / nt2, c = t0 + idx % nt2;
                    if (c < r) continue;
                    double acc = M[r * LP + c];
#pragma unroll
                    for (int k = 0; k < 16; ++k) acc = fma(-M[(j0 + k) * LP + r], M[(j0 + k) * LP + c], acc);
                    M[r * LP + c] = acc;
                }
                for (int idx = tid; idx < J * 256; idx += 1024) {
                    const int I = idx >> 8, i = (idx >> 4) & 15, c = idx & 15;
                    double acc = 0.0;
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        if (k > c) continue;
                        const double y = (k == c) ? inv_r[j0 + c] : M[(j0 + c) * LP + j0 + k];   // R_JJ^{-1}[k][c]
                        acc = fma(T[(I * 16 + i) * 16 + k], y, acc);
                    }
                    M[(j0 + c) * LP + 16 * I + i] = -acc;
                }
            }
            __syncthreads();
        }
        broke = s_broke != 0;
        __syncthreads();
        if (!broke || mode != 2) break;
        shift = (shift == 0.0) ? gmax * 0x1.0p-40 : shift * 1024.0;
        if (!(shift > 0.0)) shift = 0x1.0p-1000;
    }
    if (!broke) {
#pragma unroll 4
        for (int idx = tid; idx < L * L; idx += 1024) {
            const int x = idx / L, y = idx - x * L;
            double r = 0.0, ri = 0.0;
            if (x < l && y < l) {
                if (y >= x) r = M[x * LP + y];
                if (x <= y) ri = (x == y) ? inv_r[x] : M[y * LP + x];
            }
            R[idx] = r;
            Rinv[idx] = ri;
        }
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

hipError_t launch_chol(const double* partials, int64_t rows, int l, int L, double* R, double* Rinv, DevFlags* flags,
                       int mode, double* shift_out, double* work, double tau, hipStream_t s) {
    const int nchunks = gram_chunks(rows);
    if (l <= kCholLdsMax)
        hipLaunchKernelGGL(chol_blocked_kernel, dim3(1), dim3(1024), 0, s, partials, nchunks, l, L, R, Rinv, flags,
                           mode, shift_out, tau);
    else
        hipLaunchKernelGGL(chol_kernel<false>, dim3(1), dim3(1024), 0, s, partials, nchunks, l, L, R, Rinv, flags,
                           mode, shift_out, work, tau);
    return hipGetLastError();
}

// --------------------------------------------------------------- apply --
// out = in * M with FP64 arithmetic on FP64 MFMA (16x16x4): the CholeskyQR
// products Y R^{-1}, and the lifts U = Q U~ and V = B^T U~ Sigma^{-1}.  A
// workgroup owns 32 rows; wavefront w owns row block w & 1 and the column
// tiles t = (w >> 1), (w >> 1) + 2, ...  The inner dimension is staged
// through LDS 16 at a time with a one-slice register prefetch.  With `upper`
// set, M is upper triangular and the zero blocks below its diagonal are
// skipped.
constexpr int kApplyRows = 32;
int apply_blocks(int64_t rows) { return (int)ceil_div(rows, kApplyRows); }

template <typename T, int CT>
__global__ __launch_bounds__(256) void apply_kernel(const T* __restrict__ in, int64_t ldi, int64_t rows, int L,
                                                    const double* __restrict__ M, int ldm, int ncols_out,
                                                    T* __restrict__ out, int64_t ldo, int transpose_out,
                                                    const double* __restrict__ colscale, const DevFlags* skip,
                                                    double* __restrict__ amax_val, int* __restrict__ amax_idx,
                                                    int upper) {
    if (skip && skip->orth_fail) return;
    constexpr int W = CT * 16;
    constexpr int NTW = (CT + 1) / 2;                  // column tiles per wavefront
    constexpr int NM = (16 * W + 255) / 256;           // M elements per thread per slice
    __shared__ double inS[kApplyRows][17];
    __shared__ double MS[16][W + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int rb = 16 * (wave & 1), tw = wave >> 1;
    const int64_t row0 = (int64_t)blockIdx.x * kApplyRows;
    doublex4 acc[NTW];
#pragma unroll
    for (int j = 0; j < NTW; ++j) acc[j] = doublex4{0, 0, 0, 0};
    double pin[2], pm[NM];
    auto fetch = [&](int a0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int idx = tid + 256 * u, rr = idx >> 4, aa = idx & 15;
            const int64_t row = row0 + rr;
            pin[u] = (row < rows && a0 + aa < L) ? (double)in[row * ldi + a0 + aa] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NM; ++u) {
            const int idx = tid + 256 * u, aa = idx / W, cc = idx % W;
            pm[u] = (idx < 16 * W && a0 + aa < L && cc < ncols_out) ? M[(int64_t)(a0 + aa) * ldm + cc] : 0.0;
        }
    };
    fetch(0);
    for (int a0 = 0; a0 < L; a0 += 16) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int idx = tid + 256 * u;
            inS[idx >> 4][idx & 15] = pin[u];
        }
#pragma unroll
        for (int u = 0; u < NM; ++u) {
            const int idx = tid + 256 * u;
            if (idx < 16 * W) MS[idx / W][idx % W] = pm[u];
        }
        __syncthreads();
        if (a0 + 16 < L) fetch(a0 + 16);
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            const double av_ = inS[rb + li][kk + lk];
#pragma unroll
            for (int j = 0; j < NTW; ++j) {
                const int t = tw + 2 * j;
                if (t >= CT) continue;
                if (upper && a0 >= 16 * (t + 1)) continue;
                acc[j] = mfma16x16x4(av_, MS[kk + lk][16 * t + li], acc[j]);
            }
        }
    }
    extern __shared__ double av_dyn[];          // kApplyRows x (W + 1), argmax only
    auto avs = [&](int rr, int col) -> double& { return av_dyn[rr * (W + 1) + col]; };
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
        const int t = tw + 2 * j;
        if (t >= CT) continue;
        const int col = 16 * t + li;
        if (col >= ncols_out) continue;
        const double sc = colscale ? colscale[col] : 1.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = rb + acc_row<double>(lk, v);
            const int64_t row = row0 + rr;
            const T val = (T)(acc[j][v] * sc);
            if (row < rows) {
                if (!transpose_out) out[row * ldo + col] = val;
                else out[(int64_t)col * ldo + row] = val;
            }
            if (amax_val) avs(rr, col) = (row < rows) ? (double)val : 0.0;
        }
    }
    if (!amax_val) return;
    __syncthreads();
    for (int col = tid; col < ncols_out; col += 256) {
        double best = -1.0, val = 0.0;
        int bi = 0;
        for (int rr = 0; rr < kApplyRows; ++rr)      // lowest row wins ties
            if (fabs(avs(rr, col)) > best) { best = fabs(avs(rr, col)); val = avs(rr, col); bi = rr; }
        amax_val[(int64_t)blockIdx.x * ncols_out + col] = val;
        amax_idx[(int64_t)blockIdx.x * ncols_out + col] = (int)(row0 + bi);
    }
}

template <typename T>
static hipError_t apply_dispatch(int CT, dim3 grid, hipStream_t s, const T* in, int64_t ldi, int64_t rows, int L,
                                 const double* M, int ldm, int ncols_out, T* out, int64_t ldo, int tr,
                                 const double* colscale, const DevFlags* skip, double* av, int* ai, int upper) {
#define RSVD_CT_CASE(N)                                                                                         \
    case N:                                                                                                     \
        hipLaunchKernelGGL((apply_kernel<T, N>), grid, dim3(256),                                               \
                           av ? (size_t)kApplyRows * (N * 16 + 1) * sizeof(double) : 0, s, in, ldi, rows, L, M,  \
                           ldm, ncols_out, out, ldo, tr, colscale, skip, av, ai, upper);                        \
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
                        const DevFlags* skip, double* av, int* ai, int upper, hipStream_t s) {
    if (rows == 0 || ncols_out == 0) return hipSuccess;
    const int CT = (int)ceil_div(ncols_out, 16);
    dim3 grid(apply_blocks(rows));
    if (dtype == 0)
        return apply_dispatch<double>(CT, grid, s, (const double*)in, ldi, rows, L, M, ldm, ncols_out, (double*)out,
                                      ldo, transpose_out, colscale, skip, av, ai, upper);
    return apply_dispatch<float>(CT, grid, s, (const float*)in, ldi, rows, L, M, ldm, ncols_out, (float*)out, ldo,
                                 transpose_out, colscale, skip, av, ai, upper);
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
