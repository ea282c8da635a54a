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
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "../../include/rsvd.h"

namespace rsvd {

// ---------------------------------------------------------------- Gram --
// Partial Gram matrices Y_c^T Y_c (FP64, on FP64 MFMA 16x16x4) for nchunks
// row chunks Y_c of Y.  Output tiles of 16 x 16 on and above the diagonal.
// A workgroup of 16 wavefronts computes one tile over one chunk: wavefront w
// takes the 4-row steps w, w + 16, ... with two accumulators (so each
// wavefront has only a few batches of loads in flight one after another),
// and the 32 accumulators are summed in a fixed order.  The chunk partials
// are summed (in chunk order) by the Cholesky kernel that consumes them, so
// no workgroup ever waits for another.
int gram_pairs(int L) {
    const int nt = (int)ceil_div(L, 16);
    return nt * (nt + 1) / 2;
}
int gram_chunks(int64_t rows) { return (int)std::min<int64_t>(8, std::max<int64_t>(1, ceil_div(rows, 1024))); }
size_t gram_partials_elems(int64_t rows, int L) { return (size_t)gram_chunks(rows) * gram_pairs(L) * 256; }

constexpr int kGramWaves = 16;

template <typename T>
__global__ __launch_bounds__(64 * kGramWaves) void gram_kernel(const T* __restrict__ Y, int64_t ldy, int64_t rows,
                                                               int L, int nchunks, double* __restrict__ part,
                                                               const int* skip) {
    if (skip && *skip) return;
    const int nt = L / 16;
    const int npairs = nt * (nt + 1) / 2;
    // chunk-fastest ids: with 8 chunks each XCD takes one chunk (the rows the
    // split-K reduce and apply kernels of the same XCD wrote; xcd_block)
    const int chunk = blockIdx.x % nchunks;
    const int pair = blockIdx.x / nchunks;
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
    constexpr int STEP = 4 * kGramWaves;
    const int64_t range = r1 * ldy * (int64_t)sizeof(T);
    // every lane and scalar offset below stays under 2^31
    if (range + (int64_t)STEP * 16 * ldy * (int64_t)sizeof(T) <= 0x7fffffff) {
        // A 1024-row chunk in one batch of loads per wavefront (each round trip
        // to Y costs about 5 us), through a buffer descriptor whose range ends
        // at row r1, so rows past the chunk read as zero with no per-load
        // guard, and the loads of a batch share one lane offset and differ by
        // a scalar offset (one address register instead of one per load).
        constexpr int UNR = 16;
        const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(Y), 0, (int)range, 0x00020000);
        const int step_bytes = (int)(STEP * ldy * (int64_t)sizeof(T));
        for (int64_t k0 = r0 + 4 * wave; k0 < r1; k0 += STEP * UNR) {
            const int oa = (int)(((k0 + lk) * ldy + a * 16 + li) * (int64_t)sizeof(T));
            const int ob = oa + (b - a) * 16 * (int)sizeof(T);
            T va[UNR], vb[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                if constexpr (sizeof(T) == 4) {
                    va[u] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(ry, oa, u * step_bytes, 0));
                    vb[u] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(ry, ob, u * step_bytes, 0));
                } else {
                    va[u] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(ry, oa, u * step_bytes, 0));
                    vb[u] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(ry, ob, u * step_bytes, 0));
                }
            }
#pragma unroll
            for (int u = 0; u < UNR; u += 2) {
                acc0 = mfma16x16x4((double)va[u], (double)vb[u], acc0);
                acc1 = mfma16x16x4((double)va[u + 1], (double)vb[u + 1], acc1);
            }
        }
    } else {
        constexpr int UNR = 8;      // 8 MFMA steps (32 rows per wavefront) per batch of loads
        for (int64_t k0 = r0 + 4 * wave; k0 < r1; k0 += STEP * UNR) {
            double va[UNR], vb[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int64_t row = k0 + STEP * u + lk;
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
    }
    // acc[v] = G[a*16 + acc_row(lk, v)][b*16 + li] restricted to this chunk.
    __shared__ double red[kGramWaves][256];
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][acc_row<double>(lk, v) * 16 + li] = acc0[v] + acc1[v];
    __syncthreads();
    if (tid < 256) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < kGramWaves; ++w) sum += red[w][tid];
        part[((size_t)chunk * npairs + pair) * 256 + tid] = sum;
    }
}

hipError_t launch_gram(int dtype, const void* Y, int64_t ldy, int64_t rows, int L, double* partials,
                       const int* skip, hipStream_t s) {
    const int nchunks = gram_chunks(rows);
    dim3 grid(nchunks * gram_pairs(L));
    if (dtype == 0)
        hipLaunchKernelGGL(gram_kernel<double>, grid, dim3(64 * kGramWaves), 0, s, (const double*)Y, ldy, rows, L,
                           nchunks, partials, skip);
    else
        hipLaunchKernelGGL(gram_kernel<float>, grid, dim3(64 * kGramWaves), 0, s, (const float*)Y, ldy, rows, L,
                           nchunks, partials, skip);
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

// Form for 128 < l <= kMaxL: blocked right-looking Cholesky, panels of 16,
// one workgroup of 16 wavefronts, the working matrix A (L x L, upper block
// triangle) in global memory, where it stays in the L2 cache.  Per panel p:
//   1. wavefront 0 factors the diagonal block A_pp = R_pp^T R_pp in registers
//      (16 pivot steps inside one wavefront, no workgroup barrier) and gets
//      R_pp^{-1} from the same row operations on an identity;
//   2. R_pq = R_pp^{-T} A_pq for the tiles right of it (FP64 MFMA);
//   3. A_qr -= R_pq^T R_pr for p < q <= r (FP64 MFMA, R_p. from LDS).
// Three barriers per panel.  R^{-1} (modes 0, 1) then comes from the block
// triangle, bottom block row first: X_ij = -R_ii^{-1} sum_{i<k<=j} R_ik X_kj.
// Padding rows and columns (l <= index < L) carry an identity block, which
// no elimination step couples to the leading l x l block; the outputs are
// zero there.  Breakdown, the first-order second pass and the mode-2 shift
// retries follow the l <= 128 form.
constexpr int kCholBlkNt = kMaxL / 16;
constexpr int kCholBlkLd = kMaxL + 4;          // LDS panel row stride (doubles)

// 1 / sqrt(x) for a positive normal x: the hardware estimate and two Newton
// steps (each squares the relative error), about one ulp.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) y = fma(0.5 * y, fma(-(x * y), y, 1.0), y);
    return y;
}

// Cholesky of a 16 x 16 diagonal tile T of the augmented matrix [T | I] by
// one wavefront: lane = 16 q + c holds rows 4q .. 4q + 3 of column c of T
// (xg, upper triangle) and of the identity (xi), which the same row
// operations turn into R^{-T}.  Pivot j subtracts T[j][i] T[j][c] / d_j from
// entry (i, c) of every row i > j and then scales row j by d_j^{-1/2}.  Row j
// (its 32 entries, written by the lanes that hold it) reaches every lane
// through LDS: each lane reads the pivot, its own column's entries and its
// four rows' entries.  A wavefront's LDS operations complete in issue order,
// so the reads see the writes; the wave barrier only keeps the compiler from
// moving them.  rowbuf: 16 x 32 doubles, 16-byte aligned.  The pivots are
// tested on the way, without a branch on the chain (a bad pivot only spoils
// the steps after it): the result is true when pivot j < nvalid is not
// positive, not finite or not above rel (dgj[j] + shift) (dgj: the diagonal
// of G from the tile's first index).
__device__ __forceinline__ bool chol_tile16(double (&xg)[4], double (&xi)[4], double* rowbuf, const double* dgj,
                                            int nvalid, double rel, double shift) {
    const int lane = threadIdx.x & 63, c = lane & 15, q = lane >> 4;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        double* const rj = rowbuf + 32 * j;
        const bool holds = q == (j >> 2);               // this lane holds row j (entry j & 3)
        if (holds) {
            rj[c] = xg[j & 3];
            rj[16 + c] = xi[j & 3];
        }
        __builtin_amdgcn_wave_barrier();
        const double d = rj[j];
        const double2 t01 = *reinterpret_cast<const double2*>(rj + 4 * q);
        const double2 t23 = *reinterpret_cast<const double2*>(rj + 4 * q + 2);
        const double wg = rj[c], wi = rj[16 + c];
        if (j < nvalid) bad |= !(d > rel * (dgj[j] + shift)) || !(d > 0.0) || !isfinite(d);
        const double rs = rsqrt_nr(d), rd = rs * rs;
        const double ti[4] = {t01.x, t01.y, t23.x, t23.y};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const double f = (4 * q + m > j) ? ti[m] * rd : 0.0;
            xg[m] = fma(-f, wg, xg[m]);
            xi[m] = fma(-f, wi, xi[m]);
        }
        const double sc = holds ? rs : 1.0;
        xg[j & 3] *= sc;
        xi[j & 3] *= sc;
    }
    return bad;
}

// The same factorisation with the row entries broadcast by lane reads (lane c
// < 16: column c of T in x, lane 16 + c: column c of the identity; scale row
// j by d_j^{-1/2}, subtract R[j][i] times it from every row i > j).  It needs
// fewer vector registers than chol_tile16, which the 1024-thread block form
// cannot spare.
__device__ __forceinline__ double lane_bcast(double x, int src) {      // x of lane `src` (uniform), in every lane
    const int2 v = __builtin_bit_cast(int2, x);
    int2 r;
    r.x = __builtin_amdgcn_readlane(v.x, src);
    r.y = __builtin_amdgcn_readlane(v.y, src);
    return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ bool chol_tile16_lanes(double (&x)[16], const double* dgj, int nvalid, double rel,
                                                  double shift) {
    double dj[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        dj[j] = lane_bcast(x[j], j);
        x[j] *= rsqrt_nr(dj[j]);
#pragma unroll
        for (int i = j + 1; i < 16; ++i) x[i] = fma(-lane_bcast(x[j], i), x[j], x[i]);
    }
    bool bad = false;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (j < nvalid) bad |= !(dj[j] > rel * (dgj[j] + shift)) || !(dj[j] > 0.0) || !isfinite(dj[j]);
    return bad;
}

// End of a Cholesky kernel (modes 0, 1): the orth flags, and in mode 0 the
// test that decides whether the second CholeskyQR pass can still improve
// Q1 = Y R^{-1}.  Rounding in the FP64 Gram perturbs G by at most about
// rows 2^-53 |Y|^T |Y|, which leaves Q1^T Q1 - I at most about
// rows 2^-53 ||D R^{-1}||_F^2 (D = diag of the column norms of Y,
// D_ii^2 = G_ii); the Cholesky factorisation and the FP64 apply add far less.
// Below skip_tau the second pass is switched off.  R^{-1} is read back from
// global memory, where this workgroup has just written it.  Every thread of
// the workgroup calls this (block_sum has barriers).
// part: this thread's share of sum_ij G_ii Rinv_ij^2 when the kernel has
// accumulated it while writing R^{-1} (else negative: R^{-1} is read back).
__device__ void chol_finish_orth(DevFlags* flags, int mode, bool broke, const double* Rinv, const double* dg, int l,
                                 int L, double skip_scale, double skip_tau, int report, double* red,
                                 double part = -1.0) {
    bool off = broke;
    if (mode == 0 && !broke && skip_tau > 0.0) {
        double sum = part;
        if (part < 0.0) {
            __syncthreads();
            sum = 0.0;
            for (int idx = threadIdx.x; idx < L * L; idx += blockDim.x) {
                const int x = idx / L;
                if (x < l) {
                    const double v = Rinv[idx];
                    sum = fma(dg[x] * v, v, sum);
                }
            }
        }
        sum = block_sum(sum, red);
        off = skip_scale * sum <= skip_tau;
    }
    if (threadIdx.x == 0) {
        flags->orth_fail = broke ? 1 : 0;
        flags->pass2_off = off ? 1 : 0;
        if (broke && report) atomicOr(&flags->info, RSVD_INFO_ORTH_BREAKDOWN);
    }
}

__global__ __launch_bounds__(1024) void chol_blk_kernel(const double* __restrict__ part, int nchunks, int l, int L,
                                                        double* __restrict__ R, double* __restrict__ Rinv,
                                                        DevFlags* flags, int mode, double* shift_out,
                                                        double* __restrict__ A, double tau, double skip_scale,
                                                        double skip_tau, int report) {
    __shared__ double Dinv[kCholBlkNt][256];        // R_pp^{-1} of every diagonal block (row-major 16 x 16)
    __shared__ double Prow[16 * kCholBlkLd];        // the current panel rows R_p. (16 x L)
    __shared__ double dg[kMaxL];
    __shared__ double red[16];
    __shared__ unsigned long long s_emax;
    __shared__ int s_nonfinite, s_broke;
    if (mode == 1 && flags->pass2_off) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nt = L / 16, npairs = nt * (nt + 1) / 2, stride = npairs * 256;
    const int li = lane & 15, lk = lane >> 4;       // MFMA operand coordinates

    // A = upper block triangle of G (+ shift on the leading diagonal), identity
    // padding.  Chunk partials summed in chunk order; addresses are clamped so
    // that every load is unconditional and the 16 loads of a batch are in
    // flight together.
    auto load = [&](double shift) {
        double emax = 0.0;
        bool nf = false;
        for (int i0 = tid; i0 < stride; i0 += 2 * 1024) {
            double x[2][8];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int idx = min(i0 + u * 1024, stride - 1), cc = min(c, nchunks - 1);
                    x[u][c] = part[(size_t)cc * stride + idx];
                }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int idx = i0 + u * 1024;
                if (idx >= stride) break;
                const int pr = idx >> 8, e = idx & 255;
                int ta = 0, pp = pr;
                while (pp >= nt - ta) { pp -= nt - ta; ++ta; }
                const int row = ta * 16 + (e >> 4), col = (ta + pp) * 16 + (e & 15);
                double v;
                if (row < l && col < l) {
                    double sum = 0.0;
#pragma unroll
                    for (int c = 0; c < 8; ++c) sum += c < nchunks ? x[u][c] : 0.0;
                    if (row == col) {
                        dg[row] = sum;
                        if (!isfinite(sum)) nf = true;
                    }
                    double ee = fabs(sum - (row == col ? 1.0 : 0.0));
                    if (!(ee < 1e300)) ee = 1e300;
                    if (row <= col) emax = fmax(emax, ee);
                    v = sum + (row == col ? shift : 0.0);
                } else {
                    v = row == col ? 1.0 : 0.0;
                }
                A[(size_t)row * L + col] = v;
            }
        }
        if (nf) s_nonfinite = 1;
        return emax;
    };

    if (tid == 0) { s_emax = 0ull; s_nonfinite = 0; }
    __syncthreads();
    const double emax_t = load(0.0);
    if (mode == 1) atomicMax(&s_emax, (unsigned long long)__double_as_longlong(emax_t));
    __syncthreads();
    if (mode == 1 && __longlong_as_double((long long)s_emax) <= tau) {
        // Second pass: first-order factor R^{-1} = I - U, U = triu(E) - diag(E) / 2.
        for (int idx = tid; idx < L * L; idx += 1024) {
            const int a = idx / L, c = idx - a * L;
            double ri = 0.0;
            if (a <= c && c < l) {
                const double e = A[(size_t)a * L + c] - (a == c ? 1.0 : 0.0);
                ri = (a == c ? 1.0 : 0.0) - (a < c ? e : 0.5 * e);
            }
            Rinv[idx] = ri;
        }
        if (tid == 0) flags->orth_fail = 0;
        return;
    }
    const bool nonfinite = s_nonfinite != 0;
    const double rel = (mode == 0) ? 1e-12 : (mode == 1 ? 1e-2 : 0.0);
    double shift = 0.0;
    bool broke = nonfinite;
    for (int attempt = 0; attempt < (mode == 2 ? 5 : 1) && !nonfinite; ++attempt) {
        if (attempt > 0) {
            __syncthreads();
            load(shift);
        }
        if (tid == 0) s_broke = 0;
        __syncthreads();
        // 1. Diagonal block p in registers (wavefront 0), lane = column of
        // [A_pp | I] (chol_tile16_lanes); the identity half becomes R_pp^{-T}.
        auto factor_diag = [&](int p) {
            const int j0 = 16 * p, c = lane & 15;
            double x[16];
#pragma unroll
            for (int r = 0; r < 16; ++r)
                x[r] = lane < 16 ? (r <= c ? A[(size_t)(j0 + r) * L + j0 + c] : 0.0)
                                 : (lane < 32 && r == c ? 1.0 : 0.0);
            const bool bad = chol_tile16_lanes(x, dg + j0, l - j0, rel, shift);
            if (!bad) {
                if (lane < 16) {        // R_pp (upper) back into A for the mode-2 output
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if (r <= c) A[(size_t)(j0 + r) * L + j0 + c] = x[r];
                } else if (lane < 32) { // R_pp^{-1}, row-major: column c of R_pp^{-T} is its row c
#pragma unroll
                    for (int r = 0; r < 16; ++r) Dinv[p][c * 16 + r] = x[r];
                }
            } else if (lane == 0) {
                s_broke = 1;
            }
        };
        // p = -1 only factors the first diagonal block (one call site keeps
        // the register demand of a single inlined factorisation).
        for (int p = -1; p < nt && !s_broke; ++p) {
            if (p >= 0) {
                const int j0 = 16 * p;
                // 2. Panel row tiles: R_pq = R_pp^{-T} A_pq.
                for (int q = p + 1 + wid; q < nt; q += 16) {
                    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int st = 0; st < 4; ++st) {
                        const int k = 4 * st + lk;
                        acc = mfma16x16x4(Dinv[p][k * 16 + li], A[(size_t)(j0 + k) * L + q * 16 + li], acc);
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = lk + 4 * v;
                        A[(size_t)(j0 + r) * L + q * 16 + li] = acc[v];
                        Prow[r * kCholBlkLd + q * 16 + li] = acc[v];
                    }
                }
                __syncthreads();
                // 3. Trailing update of the tiles (q, r), p < q <= r.  Wavefront 0
                // takes the next diagonal tile (t = 0) and factors it at once while
                // the others share the remaining tiles (look-ahead).
                const int nr = nt - p - 1, ntr = nr * (nr + 1) / 2;
                for (int t = wid; t < (wid == 0 ? min(1, ntr) : ntr); t += wid == 0 ? 1 : 15) {
                    int qq = 0, tt = t;
                    while (tt >= nr - qq) { tt -= nr - qq; ++qq; }
                    const int q = p + 1 + qq, r = q + tt;
                    doublex4 acc;
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[v] = A[(size_t)(q * 16 + lk + 4 * v) * L + r * 16 + li];
#pragma unroll
                    for (int st = 0; st < 4; ++st) {
                        const int k = 4 * st + lk;
                        acc = mfma16x16x4(-Prow[k * kCholBlkLd + q * 16 + li], Prow[k * kCholBlkLd + r * 16 + li], acc);
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) A[(size_t)(q * 16 + lk + 4 * v) * L + r * 16 + li] = acc[v];
                }
            }
            if (wid == 0 && p + 1 < nt) {
                __threadfence_block();      // the tile's stores before its lanes read it back
                factor_diag(p + 1);
            }
            __syncthreads();
        }
        broke = s_broke != 0;
        if (!broke || mode != 2) break;
        double gmax = 0.0;                // largest diagonal entry (only on a retry)
        for (int j = 0; j < l; ++j) gmax = fmax(gmax, dg[j]);
        shift = (shift == 0.0) ? gmax * 0x1.0p-40 : shift * 1024.0;
        if (!(shift > 0.0)) shift = 0x1.0p-1000;
    }
    if (!broke) {
        if (mode == 2) {
            for (int idx = tid; idx < L * L; idx += 1024) {
                const int x = idx / L, y = idx - x * L;
                R[idx] = (x <= y && y < l) ? A[(size_t)x * L + y] : 0.0;
            }
        } else {
            // Diagonal blocks of R^{-1}, zero lower block triangle.
            for (int idx = tid; idx < L * L; idx += 1024) {
                const int x = idx / L, y = idx - x * L, bx = x >> 4, by = y >> 4;
                if (bx > by) Rinv[idx] = 0.0;
                else if (bx == by) Rinv[idx] = (x < l && y < l) ? Dinv[bx][(x & 15) * 16 + (y & 15)] : 0.0;
            }
            __syncthreads();
            for (int i = nt - 2; i >= 0; --i) {
                for (int j = i + 1 + wid; j < nt; j += 16) {
                    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
                    for (int k = i + 1; k <= j; ++k) {
#pragma unroll
                        for (int st = 0; st < 4; ++st) {
                            const int kk = 4 * st + lk;
                            acc = mfma16x16x4(A[(size_t)(i * 16 + li) * L + k * 16 + kk],
                                              Rinv[(size_t)(k * 16 + kk) * L + j * 16 + li], acc);
                        }
                    }
                    // The accumulator layout (rows lk + 4 v) is the B-operand layout
                    // of k-step v, so acc feeds the product with R_ii^{-1} directly.
                    doublex4 out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int st = 0; st < 4; ++st) out = mfma16x16x4(Dinv[i][li * 16 + 4 * st + lk], acc[st], out);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int x = i * 16 + lk + 4 * v, y = j * 16 + li;
                        Rinv[(size_t)x * L + y] = (x < l && y < l) ? -out[v] : 0.0;
                    }
                }
                __syncthreads();
            }
        }
    }
    if (mode != 2) chol_finish_orth(flags, mode, broke, Rinv, dg, l, L, skip_scale, skip_tau, report, red);
    if (tid == 0) {
        if (mode == 2) {
            *shift_out = shift;
            if (shift > 0.0) atomicOr(&flags->info, RSVD_INFO_SHIFTED_CHOLESKY);
            if (broke) atomicOr(&flags->info, RSVD_INFO_NONFINITE);
        }
        if (nonfinite) atomicOr(&flags->info, RSVD_INFO_NONFINITE);
    }
}

// Form for l <= 128: right-looking LDL^T elimination of the augmented
// matrix [G | I], one workgroup barrier per pivot, with the working matrix in
// registers.  With G = L D L^T the elimination turns [G | I] into
// [D L^T | L^{-1}], and row j is final once pivot j is reached, so
//   R = D^{1/2} L^T (upper, from the left half),
//   R^{-1} = L^{-T} D^{-1/2} (from the lower triangle of the right half).
// The left half is held as 8 x 8 tiles on and above the block diagonal, the
// right half as 8 x 8 tiles on and below it, one tile per thread.  Pivot row j
// updates row r > j as  row_r -= (G'_jr / d_j) row_j  over whole tiles with
// no per-element test: entries below the diagonal of the left half are
// never read into a result, and the right half of pivot row j is exactly
// zero past column j.  After step j the owners of row j + 1 publish it to
// LDS, where it is the pivot row of the next step and, at the end, the output.
// Packed LDS row r: slot s = right column s (s <= r) or left column s - 1
// (s > r); a tile publishes its whole row with unconditional stores, so the
// right half of each diagonal block goes to a separate array RD (the left
// diagonal tile's unused entries land in the packed slots it shadows).
constexpr int kCholThreads = 512;
constexpr int kCholT = 6;                         // tile edge: 2 * nb (nb + 1) / 2 <= 512 threads for l <= 128

__global__ __launch_bounds__(kCholThreads) void chol_rl_kernel(const double* __restrict__ part, int nchunks, int l,
                                                               int L, double* __restrict__ R,
                                                               double* __restrict__ Rinv, DevFlags* flags, int mode,
                                                               double* shift_out, double tau, double skip_scale,
                                                               double skip_tau, int report) {
    constexpr int T = kCholT, NBM = (kCholLdsMax + kCholT - 1) / kCholT;
    // Row stride: slots up to NBM * T (the padded tile columns), odd for bank spread.
    constexpr int LP = NBM * T + 1;
    static_assert(LP > kCholLdsMax && (LP & 1), "LDS row stride");
    __shared__ double P[kCholLdsMax * LP];        // G (upper triangle) on entry, then the packed pivot rows
    __shared__ double RD[NBM * T * T];            // right half of the diagonal blocks: RD[blk][a][b]
    __shared__ double dg[kCholLdsMax];
    __shared__ double isd[kCholLdsMax];           // D_j^{-1/2}
    __shared__ double red[kCholThreads / 64];
    __shared__ unsigned long long s_emax;
    __shared__ int s_nonfinite;
    if (mode == 1 && flags->pass2_off) return;
    const int tid = threadIdx.x;
    const int nt = L / 16, npairs = nt * (nt + 1) / 2, stride = npairs * 256;
    // Tile of this thread: tid < ntri -> left tile (bi, bj), bj >= bi; then right tile (bi, bj), bj <= bi.
    const int nb = (l + T - 1) / T, ntri = nb * (nb + 1) / 2;
    const bool owner = tid < 2 * ntri;
    const bool left = tid < ntri;
    int bi = 0, bj = 0;
    {
        int q = left ? tid : tid - ntri;
        if (!owner) q = 0;
        while (q >= nb - bi) { q -= nb - bi; ++bi; }      // row-major enumeration of the upper block triangle
        bj = bi + q;
        if (!left) { const int t = bi; bi = bj; bj = t; }
    }
    const int r0 = bi * T, c0 = bj * T;

    // Sum the chunk partials in chunk order into the upper triangle of G.
    // Addresses are clamped so that every load is unconditional and the 32
    // loads of a batch are in flight together.
    auto load = [&](double shift) {
        double emax = 0.0;
        bool nf = false;
        for (int i0 = tid; i0 < stride; i0 += 4 * kCholThreads) {
            double x[4][8];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int idx = min(i0 + u * kCholThreads, stride - 1), cc = min(c, nchunks - 1);
                    x[u][c] = part[(size_t)cc * stride + idx];
                }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = i0 + u * kCholThreads;
                if (idx >= stride) break;        // pr < npairs below keeps the pair decode finite
                double sum = 0.0;
#pragma unroll
                for (int c = 0; c < 8; ++c) sum += c < nchunks ? x[u][c] : 0.0;
                const int pr = idx >> 8, e = idx & 255;
                int ta = 0, pp = pr;
                while (pp >= nt - ta) { pp -= nt - ta; ++ta; }
                const int row = ta * 16 + (e >> 4), col = (ta + pp) * 16 + (e & 15);
                if (row > col || col >= l) continue;
                if (row == col) {
                    dg[row] = sum;
                    if (!isfinite(sum)) nf = true;
                }
                P[row * LP + col] = sum + (row == col ? shift : 0.0);
                double ee = fabs(sum - (row == col ? 1.0 : 0.0));
                if (!(ee < 1e300)) ee = 1e300;
                emax = fmax(emax, ee);
            }
        }
        if (nf) s_nonfinite = 1;
        return emax;
    };

    if (tid == 0) { s_emax = 0ull; s_nonfinite = 0; }
    __syncthreads();
    const double emax_t = load(0.0);
    if (mode == 1) atomicMax(&s_emax, (unsigned long long)__double_as_longlong(emax_t));
    __syncthreads();
    const int q4 = tid >> 7, y = tid & 127;          // output: 4 row groups of 128 columns
    if (mode == 1 && __longlong_as_double((long long)s_emax) <= tau) {
        for (int x = q4; x < L; x += 4) {
            if (y >= L) continue;
            double ri = 0.0;
            if (x <= y && y < l) {
                const double e = P[x * LP + y] - (x == y ? 1.0 : 0.0);
                ri = (x == y ? 1.0 : 0.0) - (x < y ? e : 0.5 * e);
            }
            Rinv[x * L + y] = ri;
        }
        if (tid == 0) flags->orth_fail = 0;
        return;
    }
    const bool nonfinite = s_nonfinite != 0;
    const double rel = (mode == 0) ? 1e-12 : (mode == 1 ? 1e-2 : 0.0);
    // Where this tile publishes its rows: base + a * pst + b.
    const bool rdiag = !left && bi == bj;
    double* const pub = rdiag ? RD + bi * T * T : P + r0 * LP + c0 + (left ? 1 : 0);
    const int pst = rdiag ? T : LP;
    double shift = 0.0;
    bool broke = nonfinite;
    for (int attempt = 0; attempt < (mode == 2 ? 5 : 1) && !nonfinite; ++attempt) {
        if (attempt > 0) {                // the elimination overwrote G: reload it with the new shift
            __syncthreads();
            load(shift);
            __syncthreads();
        }
        double v[T][T];
#pragma unroll
        for (int a = 0; a < T; ++a)
#pragma unroll
            for (int b = 0; b < T; ++b) {
                // Rows and columns past l hold whatever the LDS holds there;
                // they never reach a pivot row or an output.
                const int r = r0 + a, c = c0 + b;
                v[a][b] = left ? P[min(min(r, c), kCholLdsMax - 1) * LP + min(max(r, c), LP - 1)] : (r == c ? 1.0 : 0.0);
            }
        __syncthreads();                  // every read of G precedes the first pivot row written over it
        auto publish = [&](int a) {
            double* const dst = pub + a * pst;
#pragma unroll
            for (int b = 0; b < T; ++b) dst[b] = v[a][b];
        };
        if (owner && r0 == 0) publish(0);
        __syncthreads();
        // Pivots in blocks of T with the inner loop unrolled, so the tile row
        // published after step j (row j + 1) is a compile-time index.
        broke = false;
        for (int jb = 0; jb < nb && !broke; ++jb) {
#pragma unroll
            for (int jj = 0; jj < T; ++jj) {
                const int j = jb * T + jj;
                if (j >= l) break;
                const double d = P[j * LP + j + 1];
                if (!(d > rel * (dg[j] + shift)) || !(d > 0.0) || !isfinite(d)) {    // same value in every thread
                    broke = true;
                    break;
                }
                // Rows of this tile below the pivot; a right tile also needs a column <= j.
                if (owner && r0 + T - 1 > j && (left || c0 <= j)) {
                    const double* const prow = P + j * LP;
                    const double* const psrc = left ? prow + c0 + 1 : (bj == jb ? RD + jb * T * T + jj * T : prow + c0);
                    double f[T], pv[T];
#pragma unroll
                    for (int a = 0; a < T; ++a) f[a] = prow[r0 + 1 + a];
#pragma unroll
                    for (int b = 0; b < T; ++b) pv[b] = psrc[b];
                    const double rd = 1.0 / d;
#pragma unroll
                    for (int a = 0; a < T; ++a) f[a] = (r0 + a > j) ? f[a] * rd : 0.0;
#pragma unroll
                    for (int a = 0; a < T; ++a)
#pragma unroll
                        for (int b = 0; b < T; ++b) v[a][b] = fma(-f[a], pv[b], v[a][b]);
                }
                // Publish row j + 1 (also from a tile that had nothing to update).
                if (owner && j + 1 < l) {
                    if (jj < T - 1) {
                        if (jb == bi) publish(jj + 1);
                    } else if (jb + 1 == bi) {
                        publish(0);
                    }
                }
                __syncthreads();
            }
        }
        if (!broke || mode != 2) break;
        double gmax = 0.0;                // largest diagonal entry (only on a retry)
        for (int j = 0; j < l; ++j) gmax = fmax(gmax, dg[j]);
        shift = (shift == 0.0) ? gmax * 0x1.0p-40 : shift * 1024.0;
        if (!(shift > 0.0)) shift = 0x1.0p-1000;
    }
    if (!broke) {
        for (int j = tid; j < l; j += kCholThreads) isd[j] = 1.0 / sqrt(P[j * LP + j + 1]);
        __syncthreads();
        // mode 2 consumes R (the small SVD), modes 0 and 1 consume R^{-1}.
        double* out = mode == 2 ? R : Rinv;
        for (int x = q4; x < L; x += 4) {
            if (y >= L) continue;
            double val = 0.0;
            if (x <= y && y < l) {
                if (mode == 2) val = P[x * LP + y + 1] * isd[x];
                else val = ((x / T == y / T) ? RD[(y / T) * T * T + (y % T) * T + x % T] : P[y * LP + x]) * isd[y];
            }
            out[x * L + y] = val;
        }
    }
    if (mode != 2) chol_finish_orth(flags, mode, broke, Rinv, dg, l, L, skip_scale, skip_tau, report, red);
    if (tid == 0) {
        if (mode == 2) {
            *shift_out = shift;
            if (shift > 0.0) atomicOr(&flags->info, RSVD_INFO_SHIFTED_CHOLESKY);
            if (broke) atomicOr(&flags->info, RSVD_INFO_NONFINITE);
        }
        if (nonfinite) atomicOr(&flags->info, RSVD_INFO_NONFINITE);
    }
}

// Form for L <= 112 (at most 7 tiles of 16): blocked right-looking
// factorisation of the augmented matrix [G | I] with everything in LDS: the
// upper block triangle of G (left tiles) and the lower block triangle of the
// right half M.  For each block row p:
//   1. one wavefront factors the diagonal tile, G_pp = R_pp^T R_pp, in
//      registers: lane c < 16 holds column c of the tile and lane 16 + c
//      column c of the identity; pivot j scales row j by d_j^{-1/2} and
//      subtracts R_pp[j][i] times it from every row i > j, the row entries
//      broadcast by lane reads (no LDS traffic, no barrier).  The same row
//      operations turn the identity into R_pp^{-T};
//   2. block row p is multiplied by R_pp^{-T}: its left tiles become the
//      panel R_pq, its right tiles (c < p) rows of R^{-T} (FP64 MFMA);
//   3. every later block row q subtracts R_pq^T times block row p: left
//      tiles G_qr (q <= r), right tiles M_qc (c <= p) (FP64 MFMA).
// Wavefront 0 updates the next diagonal tile first and factors it while
// the others finish step 3 (look-ahead), so each block row costs two
// barriers, against one per pivot in the per-pivot form.  At the end the left tiles hold R and the right tiles R^{-T}.
// Padding rows and columns (l <= index < L) carry an identity, which no step
// couples to the leading l x l block.  Breakdown, the first-order second
// pass and the mode-2 shift retries follow the per-pivot form; mode 2 (R
// only) keeps just the diagonal right tiles R_pp^{-T}, which step 2 needs.
constexpr int kCholMfmaMaxNt = 7;
constexpr int kTileLd = 17;                    // LDS row stride of a tile (odd: conflict-free operand reads)
constexpr int kTileSz = 16 * kTileLd;

__global__ __launch_bounds__(kCholThreads) void chol_mfma_kernel(const double* __restrict__ part, int nchunks, int l,
                                                                 int L, double* __restrict__ R,
                                                                 double* __restrict__ Rinv, DevFlags* flags, int mode,
                                                                 double* shift_out, double tau, double skip_scale,
                                                                 double skip_tau, int report) {
    constexpr int NTT = kCholMfmaMaxNt * (kCholMfmaMaxNt + 1) / 2;
    __shared__ double Gt[NTT * kTileSz];        // left tiles (a, b), a <= b
    __shared__ double Mt[NTT * kTileSz];        // right tiles (q, c), c <= q
    __shared__ double dg[16 * kCholMfmaMaxNt];
    __shared__ __align__(16) double rowbuf[16 * 32];  // pivot rows of a diagonal tile
    __shared__ double red[kCholThreads / 64];
    __shared__ unsigned long long s_emax;
    __shared__ int s_nonfinite, s_broke;
    if (mode == 1 && flags->pass2_off) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = kCholThreads / 64;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = L / 16, npairs = nt * (nt + 1) / 2, stride = npairs * 256;
    auto gt = [&](int a, int b) { return Gt + (a * nt - a * (a - 1) / 2 + (b - a)) * kTileSz; };
    auto mt = [&](int q, int c) { return Mt + (q * (q + 1) / 2 + c) * kTileSz; };

    // Sum the chunk partials in chunk order into the left tiles (identity
    // outside the leading l x l block), 32 loads of a thread in flight.
    auto load = [&](double shift) {
        double emax = 0.0;
        bool nf = false;
        for (int i0 = tid; i0 < stride; i0 += 4 * kCholThreads) {
            double x[4][8];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int idx = min(i0 + u * kCholThreads, stride - 1), cc = min(c, nchunks - 1);
                    x[u][c] = part[(size_t)cc * stride + idx];
                }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = i0 + u * kCholThreads;
                if (idx >= stride) break;
                double sum = 0.0;
#pragma unroll
                for (int c = 0; c < 8; ++c) sum += c < nchunks ? x[u][c] : 0.0;
                const int pr = idx >> 8, e = idx & 255;
                int ta = 0, pp = pr;
                while (pp >= nt - ta) { pp -= nt - ta; ++ta; }
                const int row = ta * 16 + (e >> 4), col = (ta + pp) * 16 + (e & 15);
                double v;
                if (row < l && col < l) {
                    if (row == col) {
                        dg[row] = sum;
                        if (!isfinite(sum)) nf = true;
                    }
                    if (row <= col) {
                        double ee = fabs(sum - (row == col ? 1.0 : 0.0));
                        if (!(ee < 1e300)) ee = 1e300;
                        emax = fmax(emax, ee);
                    }
                    v = sum + (row == col ? shift : 0.0);
                } else {
                    v = row == col ? 1.0 : 0.0;
                }
                gt(ta, ta + pp)[(e >> 4) * kTileLd + (e & 15)] = v;
            }
        }
        if (nf) s_nonfinite = 1;
        return emax;
    };

    if (tid == 0) { s_emax = 0ull; s_nonfinite = 0; }
    __syncthreads();
    const double emax_t = load(0.0);
    if (mode == 1) atomicMax(&s_emax, (unsigned long long)__double_as_longlong(emax_t));
    __syncthreads();
    if (mode == 1 && __longlong_as_double((long long)s_emax) <= tau) {
        // Second pass: first-order factor R^{-1} = I - U, U = triu(E) - diag(E) / 2.
        for (int x = wid; x < L; x += nw)
            for (int y = lane; y < L; y += 64) {
                double ri = 0.0;
                if (x <= y && y < l) {
                    const double e = gt(x >> 4, y >> 4)[(x & 15) * kTileLd + (y & 15)] - (x == y ? 1.0 : 0.0);
                    ri = (x == y ? 1.0 : 0.0) - (x < y ? e : 0.5 * e);
                }
                Rinv[x * L + y] = ri;
            }
        if (tid == 0) flags->orth_fail = 0;
        return;
    }
    const bool nonfinite = s_nonfinite != 0;
    const double rel = (mode == 0) ? 1e-12 : (mode == 1 ? 1e-2 : 0.0);
    const bool inv = mode != 2;                 // R^{-1} wanted: the whole right half
    double shift = 0.0;
    bool broke = nonfinite;
    for (int attempt = 0; attempt < (mode == 2 ? 5 : 1) && !nonfinite; ++attempt) {
        if (attempt > 0) {                // the elimination overwrote G: reload it with the new shift
            __syncthreads();
            load(shift);
        }
        if (inv)
            for (int idx = tid; idx < NTT * kTileSz; idx += kCholThreads) Mt[idx] = 0.0;
        if (tid == 0) s_broke = 0;
        __syncthreads();
        // 1. Diagonal tile p of [G_pp | I] in registers (wavefront 0,
        // chol_tile16): a bad pivot only spoils the steps after it, which
        // are then discarded.
        auto factor_diag = [&](int p) {
            double* const T = gt(p, p);
            const int c = lane & 15, r0 = 4 * (lane >> 4);
            double xg[4], xi[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                xg[m] = r0 + m <= c ? T[(r0 + m) * kTileLd + c] : 0.0;
                xi[m] = r0 + m == c ? 1.0 : 0.0;
            }
            const bool bad = chol_tile16(xg, xi, rowbuf, dg + 16 * p, l - 16 * p, rel, shift);
            if (!bad) {
                double* const D = mt(p, p);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    T[(r0 + m) * kTileLd + c] = r0 + m <= c ? xg[m] : 0.0;
                    D[(r0 + m) * kTileLd + c] = xi[m];
                }
            } else if (lane == 0) {
                s_broke = 1;
            }
        };
        if (wid == 0) factor_diag(0);
        __syncthreads();
        for (int p = 0; p < nt && !s_broke; ++p) {
            // 2. Block row p times R_pp^{-T}: left tiles q > p, right tiles c < p.
            const int nleft = nt - p - 1, nright = inv ? p : 0;
            const double* const Dp = mt(p, p);
            for (int jb = wid; jb < nleft + nright; jb += nw) {
                double* const B = jb < nleft ? gt(p, p + 1 + jb) : mt(p, jb - nleft);
                doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const int k = 4 * st + lk;
                    acc = mfma16x16x4(Dp[li * kTileLd + k], B[k * kTileLd + li], acc);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) B[(lk + 4 * v) * kTileLd + li] = acc[v];
            }
            __syncthreads();
            // 3. Trailing update of the later block rows.  Wavefront 0 takes
            // the next diagonal tile (the first job) and factors it at once,
            // while the others share the remaining jobs (look-ahead).
            const int nq = nt - p - 1, nl = nq * (nq + 1) / 2, nr = inv ? nq * (p + 1) : 0;
            for (int jb = wid == 0 ? 0 : wid; jb < (wid == 0 ? min(1, nl) : nl + nr); jb += nw - 1) {
                const double* Aop;
                const double* Bop;
                double* C;
                if (jb < nl) {
                    int qq = 0, tt = jb;
                    while (tt >= nq - qq) { tt -= nq - qq; ++qq; }
                    const int q = p + 1 + qq, r = q + tt;
                    Aop = gt(p, q);
                    Bop = gt(p, r);
                    C = gt(q, r);
                } else {
                    const int j2 = jb - nl, q = p + 1 + j2 / (p + 1), c = j2 % (p + 1);
                    Aop = gt(p, q);
                    Bop = mt(p, c);
                    C = mt(q, c);
                }
                doublex4 acc;
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] = C[(lk + 4 * v) * kTileLd + li];
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const int k = 4 * st + lk;
                    acc = mfma16x16x4(-Aop[k * kTileLd + li], Bop[k * kTileLd + li], acc);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) C[(lk + 4 * v) * kTileLd + li] = acc[v];
            }
            if (wid == 0 && p + 1 < nt) factor_diag(p + 1);
            __syncthreads();
        }
        broke = s_broke != 0;
        if (!broke || mode != 2) break;
        double gmax = 0.0;                // largest diagonal entry (only on a retry)
        for (int j = 0; j < l; ++j) gmax = fmax(gmax, dg[j]);
        shift = (shift == 0.0) ? gmax * 0x1.0p-40 : shift * 1024.0;
        if (!(shift > 0.0)) shift = 0x1.0p-1000;
    }
    double ssum = 0.0;                          // sum of G_ii Rinv_ij^2 over this thread's entries
    if (!broke) {
        for (int x = wid; x < L; x += nw) {
            const double dgx = x < l ? dg[x] : 0.0;
            for (int y = lane; y < L; y += 64) {
                const bool in = x <= y && y < l;
                if (mode == 2) {
                    R[x * L + y] = in ? gt(x >> 4, y >> 4)[(x & 15) * kTileLd + (y & 15)] : 0.0;
                } else {
                    const double v = in ? mt(y >> 4, x >> 4)[(y & 15) * kTileLd + (x & 15)] : 0.0;
                    Rinv[x * L + y] = v;
                    ssum = fma(dgx * v, v, ssum);
                }
            }
        }
    }
    if (mode != 2) chol_finish_orth(flags, mode, broke, Rinv, dg, l, L, skip_scale, skip_tau, report, red, ssum);
    if (tid == 0) {
        if (mode == 2) {
            *shift_out = shift;
            if (shift > 0.0) atomicOr(&flags->info, RSVD_INFO_SHIFTED_CHOLESKY);
            if (broke) atomicOr(&flags->info, RSVD_INFO_NONFINITE);
        }
        if (nonfinite) atomicOr(&flags->info, RSVD_INFO_NONFINITE);
    }
}

hipError_t launch_chol(const double* partials, int64_t rows, int l, int L, double* R, double* Rinv, DevFlags* flags,
                       int mode, double* shift_out, double* work, double tau, hipStream_t s, double skip_tau,
                       int report_breakdown) {
    const int nchunks = gram_chunks(rows);
    const double skip_scale = (double)rows * 0x1.0p-53;
    if (L <= 16 * kCholMfmaMaxNt)
        hipLaunchKernelGGL(chol_mfma_kernel, dim3(1), dim3(kCholThreads), 0, s, partials, nchunks, l, L, R, Rinv, flags,
                           mode, shift_out, tau, skip_scale, skip_tau, report_breakdown);
    else if (l <= kCholLdsMax)
        hipLaunchKernelGGL(chol_rl_kernel, dim3(1), dim3(kCholThreads), 0, s, partials, nchunks, l, L, R, Rinv, flags,
                           mode, shift_out, tau, skip_scale, skip_tau, report_breakdown);
    else
        hipLaunchKernelGGL(chol_blk_kernel, dim3(1), dim3(1024), 0, s, partials, nchunks, l, L, R, Rinv, flags,
                           mode, shift_out, work, tau, skip_scale, skip_tau, report_breakdown);
    return hipGetLastError();
}

// --------------------------------------------------------------- apply --
// out = in * M with FP64 arithmetic on FP64 MFMA (16x16x4): the CholeskyQR
// products Y R^{-1}, and the lifts U = Q U~ and V = B^T U~ Sigma^{-1}.  A
// workgroup owns 32 rows; wavefront w owns row block w & 1 and the column
// tiles t = (w >> 1), (w >> 1) + 2, ...  The inner dimension is staged
// through LDS 16 at a time with a one-slice register prefetch.  With `upper`
// set, M is upper triangular and this form skips the zero blocks below its
// diagonal (the LDS form below multiplies them).
constexpr int kApplyRows = 32;
int apply_blocks(int64_t rows) { return (int)ceil_div(rows, kApplyRows); }

template <typename T, int CT>
__global__ __launch_bounds__(256) void apply_kernel(const T* in, int64_t ldi, int64_t rows, int L,
                                                    const double* __restrict__ M, int ldm, int ncols_out,
                                                    T* out, int64_t ldo, int transpose_out,
                                                    const double* __restrict__ colscale, const int* skip,
                                                    double* __restrict__ amax_val, int* __restrict__ amax_idx,
                                                    int upper) {
    if (skip && *skip) return;
    constexpr int W = CT * 16;
    constexpr int NTW = (CT + 1) / 2;                  // column tiles per wavefront
    constexpr int NM = (16 * W + 255) / 256;           // M elements per thread per slice
    __shared__ double inS[kApplyRows][17];
    __shared__ double MS[16][W + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int rb = 16 * (wave & 1), tw = wave >> 1;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row0 = blk * kApplyRows;
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
        amax_val[blk * ncols_out + col] = val;
        amax_idx[blk * ncols_out + col] = (int)(row0 + bi);
    }
}

// Variant for L <= 128 and at most 112 output columns (LDS: 32 x 129 + 128 x
// 113 doubles): the workgroup's 32
// rows of `in` and all of M are loaded into LDS at once (every load in
// flight together), then the products run as above.  The argmax partials
// reuse the LDS of the input rows.
constexpr int kApplyLdsMax = 128;

template <typename T, int CT>
__global__ __launch_bounds__(256) void apply_lds_kernel(const T* in, int64_t ldi, int64_t rows, int L,
                                                        const double* __restrict__ M, int ldm, int ncols_out,
                                                        T* out, int64_t ldo, int transpose_out,
                                                        const double* __restrict__ colscale, const int* skip,
                                                        double* __restrict__ amax_val, int* __restrict__ amax_idx,
                                                        int upper) {
    if (skip && *skip) return;
    constexpr int W = CT * 16;
    constexpr int NTW = (CT + 1) / 2;
    constexpr int SI = kApplyLdsMax + 1;               // row stride of the input rows (odd)
    constexpr int SM = W + 1;
    static_assert(kApplyRows * SI >= kApplyRows * SM, "argmax partials reuse the input rows' LDS");
    __shared__ double inS[kApplyRows * SI];
    __shared__ double MS[kApplyLdsMax * SM];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int rb = 16 * (wave & 1), tw = wave >> 1;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row0 = blk * kApplyRows;
    // Input rows (16-byte vectors of `in`) and M (pairs of doubles), every
    // load of the thread issued before the first store.  L and W are
    // multiples of 16, the leading dimensions multiples of 16 elements and
    // the buffers 16-byte aligned (internal panels and workspace).
    {
        constexpr int VI = 16 / (int)sizeof(T);                       // elements per vector of `in`
        constexpr int NI = (kApplyRows * kApplyLdsMax / VI + 255) / 256;
        constexpr int NV = (kApplyLdsMax * W / 2 + 255) / 256;
        using VT = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
        VT vi[NI];
        double2 vm[NV];
        const int ni = kApplyRows * L / VI, nm = L * W / 2;
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int idx = min(tid + 256 * u, ni - 1), rr = idx / (L / VI), aa = (idx - rr * (L / VI)) * VI;
            const int64_t row = min(row0 + rr, rows - 1);              // rows past the end are never stored
            vi[u] = *reinterpret_cast<const VT*>(in + row * ldi + aa);
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const int idx = min(tid + 256 * u, nm - 1), aa = idx / (W / 2), cc = (idx - aa * (W / 2)) * 2;
            vm[u] = *reinterpret_cast<const double2*>(M + (int64_t)aa * ldm + min(cc, ldm - 2));
        }
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int idx = tid + 256 * u, rr = idx / (L / VI), aa = (idx - rr * (L / VI)) * VI;
            if (idx < ni) {
#pragma unroll
                for (int e = 0; e < VI; ++e) {
                    double x;
                    if constexpr (sizeof(T) == 4) x = e == 0 ? vi[u].x : e == 1 ? vi[u].y : e == 2 ? vi[u].z : vi[u].w;
                    else x = e == 0 ? vi[u].x : vi[u].y;
                    inS[rr * SI + aa + e] = row0 + rr < rows ? x : 0.0;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const int idx = tid + 256 * u, aa = idx / (W / 2), cc = (idx - aa * (W / 2)) * 2;
            if (idx < nm) {
                MS[aa * SM + cc] = cc < ncols_out ? vm[u].x : 0.0;
                MS[aa * SM + cc + 1] = cc + 1 < ncols_out ? vm[u].y : 0.0;
            }
        }
    }
    __syncthreads();
    doublex4 acc[NTW];
#pragma unroll
    for (int j = 0; j < NTW; ++j) acc[j] = doublex4{0, 0, 0, 0};
    // Per 16-deep K block, the operand fragments (4 MFMA steps x the wave's
    // column tiles) are read from LDS together, then the matrix instructions
    // run back to back.  The loop has no branch: a tile past CT reads a
    // clamped column and is never stored, and with `upper` the zero blocks of
    // M below its diagonal are multiplied like the others (at L <= 128,
    // skipping them per tile put a branch around every matrix instruction,
    // which then waited for its result before the next: 2.3 times slower).
    (void)upper;
    for (int a0 = 0; a0 < L; a0 += 16) {
        double av[4], bv[NTW][4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = a0 + 4 * kk + lk;
            av[kk] = inS[(rb + li) * SI + k];
#pragma unroll
            for (int j = 0; j < NTW; ++j) bv[j][kk] = MS[k * SM + min(16 * (tw + 2 * j), W - 16) + li];
        }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int j = 0; j < NTW; ++j) acc[j] = mfma16x16x4(av[kk], bv[j][kk], acc[j]);
    }
    if (amax_val) __syncthreads();                     // the input rows' LDS becomes the argmax scratch
    auto avs = [&](int rr, int col) -> double& { return inS[rr * SM + col]; };
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
        amax_val[blk * ncols_out + col] = val;
        amax_idx[blk * ncols_out + col] = (int)(row0 + bi);
    }
}

template <typename T>
static hipError_t apply_lds_dispatch(int CT, dim3 grid, hipStream_t s, const T* in, int64_t ldi, int64_t rows, int L,
                                     const double* M, int ldm, int ncols_out, T* out, int64_t ldo, int tr,
                                     const double* colscale, const int* skip, double* av, int* ai, int upper) {
#define RSVD_CT_CASE(N)                                                                                          \
    case N:                                                                                                      \
        hipLaunchKernelGGL((apply_lds_kernel<T, N>), grid, dim3(256), 0, s, in, ldi, rows, L, M, ldm, ncols_out,  \
                           out, ldo, tr, colscale, skip, av, ai, upper);                                         \
        break;
    switch (CT) {
        RSVD_CT_CASE(1) RSVD_CT_CASE(2) RSVD_CT_CASE(3) RSVD_CT_CASE(4) RSVD_CT_CASE(5) RSVD_CT_CASE(6)
        RSVD_CT_CASE(7)
        default: return hipErrorInvalidValue;
    }
#undef RSVD_CT_CASE
    return hipGetLastError();
}

template <typename T>
static hipError_t apply_dispatch(int CT, dim3 grid, hipStream_t s, const T* in, int64_t ldi, int64_t rows, int L,
                                 const double* M, int ldm, int ncols_out, T* out, int64_t ldo, int tr,
                                 const double* colscale, const int* skip, double* av, int* ai, int upper) {
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
                        const int* skip, double* av, int* ai, int upper, hipStream_t s) {
    if (rows == 0 || ncols_out == 0) return hipSuccess;
    const int CT = (int)ceil_div(ncols_out, 16);
    dim3 grid(apply_blocks(rows));
    if (L <= kApplyLdsMax && CT <= 7) {
        if (dtype == 0)
            return apply_lds_dispatch<double>(CT, grid, s, (const double*)in, ldi, rows, L, M, ldm, ncols_out,
                                              (double*)out, ldo, transpose_out, colscale, skip, av, ai, upper);
        return apply_lds_dispatch<float>(CT, grid, s, (const float*)in, ldi, rows, L, M, ldm, ncols_out, (float*)out,
                                         ldo, transpose_out, colscale, skip, av, ai, upper);
    }
    if (dtype == 0)
        return apply_dispatch<double>(CT, grid, s, (const double*)in, ldi, rows, L, M, ldm, ncols_out, (double*)out,
                                      ldo, transpose_out, colscale, skip, av, ai, upper);
    return apply_dispatch<float>(CT, grid, s, (const float*)in, ldi, rows, L, M, ldm, ncols_out, (float*)out, ldo,
                                 transpose_out, colscale, skip, av, ai, upper);
}

// ---------------------------------------------------------- Householder --
// Fallback thin QR by Householder reflections, for a Y that CholeskyQR
// cannot factor (rank-deficient, zero, or too ill-conditioned), as a TSQR
// tree on many workgroups.  Level 1 splits the rows into G1 <= 64 chunks of
// at least L rows; each workgroup factors its chunk Y_c = Q_c R_c.  Each
// higher level stacks up to 4 of the R factors below it and factors the
// stack, until one factor R remains (the root).  A stack of upper-triangular
// L x L blocks keeps that form under its own reflections, so reflector j of
// a stack touches only row j of the first block and rows 0..j of the others
// (HhRows), about a third of the stack's rows on average.  Q is then formed top down:
// the root's reflectors applied to the first l columns of the identity give
// M (a stack of L x L blocks); each tile below applies its reflectors to
// [its block of M; 0], and at level 1 that is the tile's rows of Q.  Columns
// whose root diagonal entry of R is negative are negated (diag(R) >= 0).
// All work is FP64 in device scratch: H (level-1 reflectors, rows x L),
// Qw (level-1 Q, rows x L) and `up` (the stacks and M blocks of the higher
// levels, the tau and beta vectors of every level).
//
// The levels are separated by a grid-wide barrier (one counter and one
// generation word in the flags block, counter zero between barriers), so
// the kernel is launched with one workgroup per level-1 chunk (<= 64
// workgroups of 512 threads, all resident at once on 256 compute units);
// the waits are bounded, and a barrier that does not complete sets
// RSVD_INFO_FALLBACK_TIMEOUT instead of hanging.  When the CholeskyQR
// passes succeeded (and the fallback is not forced) every workgroup returns
// at once.
constexpr int kHhThreads = 512;
constexpr int kHhMaxChunks = 64;
constexpr int kHhFanIn = 4;
constexpr int kHhMaxLevels = 4;             // 64 -> 16 -> 4 -> 1
// Reflectors of tiles up to kHhVsMax rows are staged in LDS (128 KB, one
// workgroup per compute unit); longer level-1 chunks (more than about a
// million rows) read them in place.
constexpr int kHhVsMax = 16384;

struct HhTree {
    int nlev;
    int n[kHhMaxLevels + 1];                // tiles per level (index 1..nlev)
    int64_t s_off[kHhMaxLevels + 1];        // level h >= 2: stack of level h (n[h-1] L rows, L columns)
    int64_t m_off[kHhMaxLevels + 1];        // level h >= 2: M blocks of level h (same shape)
    int64_t t_off[kHhMaxLevels + 1];        // tau of level h (n[h] L), beta follows (n[h] L)
    int64_t total;                          // doubles of `up`
};

static HhTree hh_tree(int64_t rows, int L) {
    HhTree t{};
    t.n[1] = (int)std::max<int64_t>(1, std::min<int64_t>(kHhMaxChunks, rows / L));
    t.nlev = 1;
    while (t.n[t.nlev] > 1) {
        t.n[t.nlev + 1] = (t.n[t.nlev] + kHhFanIn - 1) / kHhFanIn;
        ++t.nlev;
    }
    int64_t off = 0;
    for (int h = 2; h <= t.nlev; ++h) {
        t.s_off[h] = off;
        off += (int64_t)t.n[h - 1] * L * L;
        t.m_off[h] = off;
        off += (int64_t)t.n[h - 1] * L * L;
    }
    for (int h = 1; h <= t.nlev; ++h) {
        t.t_off[h] = off;
        off += 2 * (int64_t)t.n[h] * L;
    }
    t.total = off;
    return t;
}

size_t householder_scratch_doubles(int64_t rows, int L) { return (size_t)hh_tree(rows, L).total; }

// Bounded grid barrier for `nblocks` workgroups: the last arrival resets the
// counter and bumps the generation; agent-scope fences order every
// workgroup's global writes before the barrier with the reads after it.
__device__ void hh_grid_sync(DevFlags* flags, int nblocks) {
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned* ctr = reinterpret_cast<unsigned*>(&flags->fb_count);
        unsigned* gen = reinterpret_cast<unsigned*>(&flags->fb_gen);
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        if (atomicAdd(ctr, 1u) == (unsigned)nblocks - 1u) {
            __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(8);
                if (++spins == (1u << 24)) {              // about a second: give up, report it
                    atomicOr(&flags->info, RSVD_INFO_FALLBACK_TIMEOUT);
                    break;
                }
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// The rows of reflector j of a tile (nr rows, row stride L): rows j..nr-1 of
// a dense tile (level 1), or, in a stack of upper-triangular L x L blocks
// (the higher levels), row j of the first block and rows 0..j of each of
// the others, where every other entry of the reflector's column and of the
// columns it updates is zero.  Rows are numbered s = 0 .. count() - 1.
struct HhRows {
    int j, nr, L;
    bool stk;
    __device__ int count() const { return stk ? 1 + (nr / L - 1) * (j + 1) : nr - j; }
    __device__ int row(int s) const {
        if (!stk) return j + s;
        if (s == 0) return j;
        const int t = s - 1;
        return (1 + t / (j + 1)) * L + t % (j + 1);
    }
};

// X <- (I - tau v v^T) X on the rows rs of reflector j and columns c0..l-1
// of X (row stride L), the reflector v in v[i * vst] (in LDS with vst = 1, or
// in place in the tile with vst = L): w = tau v^T X, then X -= v w.  The
// workgroup works on 128 columns at a time, one column per lane, so every
// load and store of a row is contiguous across the lanes; the kHhThreads /
// 128 row groups take rows s = g, g + groups, ... of rs with eight loads in flight, and
// their partial inner products are summed in group order through wbuf
// (kHhThreads doubles of LDS).  Every thread of the workgroup calls this.
__device__ void hh_reflect_block(double* X, const double* v, int vst, const HhRows& rs, int c0, int l, double tj,
                                 double* wbuf) {
    constexpr int CG = 128, U = 8;
    const int tid = threadIdx.x, cl = tid % CG, rg = tid / CG, nrg = blockDim.x / CG;
    const int64_t sv = vst, L = rs.L;
    const int n = rs.count();
    for (int cb = c0; cb < l; cb += CG) {
        const int c = cb + cl;
        const bool act = c < l;
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = 0.0;
        if (act) {
            int s = rg;
            for (; s + (U - 1) * nrg < n; s += U * nrg) {
                int i[U];
                double x[U];
#pragma unroll
                for (int u = 0; u < U; ++u) i[u] = rs.row(s + u * nrg);
#pragma unroll
                for (int u = 0; u < U; ++u) x[u] = X[i[u] * L + c];
#pragma unroll
                for (int u = 0; u < U; ++u) a[u] = fma(v[i[u] * sv], x[u], a[u]);
            }
            for (; s < n; s += nrg) {
                const int i = rs.row(s);
                a[0] = fma(v[i * sv], X[i * L + c], a[0]);
            }
        }
        wbuf[rg * CG + cl] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        __syncthreads();
        double w = 0.0;
        for (int g = 0; g < nrg; ++g) w += wbuf[g * CG + cl];
        w *= tj;
        if (act) {
            int s = rg;
            for (; s + (U - 1) * nrg < n; s += U * nrg) {
                int i[U];
                double x[U];
#pragma unroll
                for (int u = 0; u < U; ++u) i[u] = rs.row(s + u * nrg);
#pragma unroll
                for (int u = 0; u < U; ++u) x[u] = X[i[u] * L + c];
#pragma unroll
                for (int u = 0; u < U; ++u) X[i[u] * L + c] = fma(-w, v[i[u] * sv], x[u]);
            }
            for (; s < n; s += nrg) {
                const int i = rs.row(s);
                X[i * L + c] = fma(-w, v[i * sv], X[i * L + c]);
            }
        }
        __syncthreads();                            // wbuf is reused by the next block of columns
    }
}

// Householder QR in place of the tile T (nr rows, row stride L, FP64): for
// column j < min(nr, l), the reflector v (v_0 on the diagonal, the rest
// below it) with tau_j = 2 / v^T v maps the trailing part of column j onto
// beta_j e_1; the trailing columns c < l are updated by the whole workgroup
// (hh_reflect_block).  Above the diagonal T then holds R; beta holds its
// diagonal.  vs: LDS for nr doubles; wbuf: LDS for blockDim.x doubles.
__device__ void hh_factor_tile(double* T, int nr, int L, int l, bool stk, double* tau, double* beta, double* red,
                               double* vs, double* wbuf) {
    const int tid = threadIdx.x;
    const int jmax = min(nr, l);
    const bool in_lds = nr <= kHhVsMax;
    for (int j = 0; j < jmax; ++j) {
        const HhRows rs{j, nr, L, stk};
        const int n = rs.count();
        double s = 0.0;
        for (int q = tid; q < n; q += blockDim.x) {
            const int i = rs.row(q);
            const double x = T[(int64_t)i * L + j];
            if (in_lds) vs[i] = x;
            s = fma(x, x, s);
        }
        s = block_sum(s, red);                      // its barriers also publish vs
        const double alpha = T[(int64_t)j * L + j];
        const double normx = sqrt(s);
        if (normx == 0.0) {
            if (tid == 0) { tau[j] = 0.0; beta[j] = 0.0; }
            __syncthreads();
            continue;
        }
        const double bj = alpha >= 0.0 ? -normx : normx;
        const double v0 = alpha - bj;
        const double tj = 2.0 / (s - alpha * alpha + v0 * v0);
        __syncthreads();
        if (tid == 0) {
            T[(int64_t)j * L + j] = v0;
            if (in_lds) vs[j] = v0;
            tau[j] = tj;
            beta[j] = bj;
        }
        __syncthreads();
        const double* v = in_lds ? vs : T + j;
        hh_reflect_block(T, v, in_lds ? 1 : L, rs, j + 1, l, tj, wbuf);
    }
}

// Z (nr x L) <- H_0 H_1 ... H_{jmax-1} Z with the reflectors of tile T (as
// left by hh_factor_tile), columns c < l only.  vs: LDS for nr doubles;
// wbuf: LDS for blockDim.x doubles.
__device__ void hh_apply_tile(const double* T, int nr, int L, int l, bool stk, const double* tau, double* Z,
                              double* vs, double* wbuf) {
    const int tid = threadIdx.x;
    const int jmax = min(nr, l);
    const bool in_lds = nr <= kHhVsMax;
    for (int j = jmax - 1; j >= 0; --j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;                    // same value in every thread
        const HhRows rs{j, nr, L, stk};
        if (in_lds)
            for (int q = tid; q < rs.count(); q += blockDim.x) {
                const int i = rs.row(q);
                vs[i] = T[(int64_t)i * L + j];
            }
        __syncthreads();
        const double* v = in_lds ? vs : T + j;
        hh_reflect_block(Z, v, in_lds ? 1 : L, rs, 0, l, tj, wbuf);
    }
}

template <typename T>
__global__ __launch_bounds__(kHhThreads) void householder_kernel(const T* __restrict__ Y, int64_t ldy, int64_t rows,
                                                                 int l, int L, T* __restrict__ Q, int64_t ldq,
                                                                 double* __restrict__ H, double* __restrict__ Qw,
                                                                 double* __restrict__ up, DevFlags* flags, int force,
                                                                 HhTree tr) {
    if (!force && !flags->orth_fail) return;
    __shared__ double red[kHhThreads / 64];
    __shared__ double vs[kHhVsMax];                 // the current reflector (tile rows <= kHhVsMax)
    __shared__ double wbuf[kHhThreads];             // partial inner products of hh_reflect_block
    const int tid = threadIdx.x, b = blockIdx.x, G = gridDim.x;
    auto chunk = [&](int c) { return (int64_t)c * rows / tr.n[1]; };     // level-1 chunk c: rows [chunk(c), chunk(c+1))
    auto tile_rows = [&](int h, int t) -> int {                           // rows of tile t at level h >= 2
        return (min(kHhFanIn * (t + 1), tr.n[h - 1]) - kHhFanIn * t) * L;
    };
    auto tile_base = [&](int h, int t) -> double* {                       // stack of level h, tile t
        return h == 1 ? H + chunk(t) * L : up + tr.s_off[h] + (int64_t)kHhFanIn * t * L * L;
    };
    auto m_base = [&](int h, int t) -> double* {                          // M of level h, tile t
        return h == 1 ? Qw + chunk(t) * L : up + tr.m_off[h] + (int64_t)kHhFanIn * t * L * L;
    };
    auto nrows = [&](int h, int t) -> int { return h == 1 ? (int)(chunk(t + 1) - chunk(t)) : tile_rows(h, t); };

    // Up the tree: factor, and pass R to the parent's stack.
    for (int h = 1; h <= tr.nlev; ++h) {
        if (b < tr.n[h]) {
            double* Tt = tile_base(h, b);
            const int nr = nrows(h, b);
            if (h == 1) {
                const int64_t r0 = chunk(b);
                for (int64_t idx = tid; idx < (int64_t)nr * L; idx += kHhThreads) {
                    const int64_t i = idx / L;
                    const int c = (int)(idx % L);
                    Tt[idx] = c < l ? (double)Y[(r0 + i) * ldy + c] : 0.0;
                }
                __syncthreads();
            }
            double* tau = up + tr.t_off[h] + (int64_t)b * L;
            double* beta = tau + (int64_t)tr.n[h] * L;
            hh_factor_tile(Tt, nr, L, l, h > 1, tau, beta, red, vs, wbuf);
            if (h < tr.nlev) {                          // R of this tile -> block b of the level h + 1 stack
                double* Rp = up + tr.s_off[h + 1] + (int64_t)b * L * L;
                for (int idx = tid; idx < L * L; idx += kHhThreads) {
                    const int x = idx / L, c = idx - x * L;
                    double v = 0.0;
                    if (x < nr && c < l) v = c == x ? beta[x] : (c > x ? Tt[(int64_t)x * L + c] : 0.0);
                    Rp[idx] = v;
                }
            }
        }
        if (h < tr.nlev) hh_grid_sync(flags, G);
    }
    // Down the tree: M of the root from the identity, then each tile's block.
    const double* beta_root = up + tr.t_off[tr.nlev] + (int64_t)tr.n[tr.nlev] * L;
    for (int h = tr.nlev; h >= 1; --h) {
        if (b < tr.n[h]) {
            const int nr = nrows(h, b);
            double* Z = m_base(h, b);
            const double* Min = h == tr.nlev ? nullptr : up + tr.m_off[h + 1] + (int64_t)b * L * L;
            for (int64_t idx = tid; idx < (int64_t)nr * L; idx += kHhThreads) {
                const int64_t i = idx / L;
                const int c = (int)(idx % L);
                double v = 0.0;
                if (i < L) v = Min ? Min[idx] : ((i == c && c < l) ? 1.0 : 0.0);
                Z[idx] = v;
            }
            __syncthreads();
            const double* tau = up + tr.t_off[h] + (int64_t)b * L;
            hh_apply_tile(tile_base(h, b), nr, L, l, h > 1, tau, Z, vs, wbuf);
            if (h == 1) {                               // this chunk's rows of Q, signs from the root's R
                const int64_t r0 = chunk(b);
                for (int64_t idx = tid; idx < (int64_t)nr * L; idx += kHhThreads) {
                    const int64_t i = idx / L;
                    const int c = (int)(idx % L);
                    Q[(r0 + i) * ldq + c] = c < l ? (T)(beta_root[c] < 0.0 ? -Z[idx] : Z[idx]) : (T)0;
                }
            }
        }
        if (h > 1) hh_grid_sync(flags, G);
    }
    if (tid == 0 && b == 0) atomicOr(&flags->info, RSVD_INFO_QR_FALLBACK);
}

hipError_t launch_householder(int dtype, const void* Y, int64_t ldy, int64_t rows, int l, int L, void* Q,
                              int64_t ldq, double* H, double* Qw, double* up, DevFlags* flags, int force,
                              hipStream_t s) {
    const HhTree tr = hh_tree(rows, L);
    dim3 grid(tr.n[1]);
    if (dtype == 0)
        hipLaunchKernelGGL(householder_kernel<double>, grid, dim3(kHhThreads), 0, s, (const double*)Y, ldy, rows, l, L,
                           (double*)Q, ldq, H, Qw, up, flags, force, tr);
    else
        hipLaunchKernelGGL(householder_kernel<float>, grid, dim3(kHhThreads), 0, s, (const float*)Y, ldy, rows, l, L,
                           (float*)Q, ldq, H, Qw, up, flags, force, tr);
    return hipGetLastError();
}

}  // namespace rsvd
