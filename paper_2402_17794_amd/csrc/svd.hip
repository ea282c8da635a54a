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
// l <= 128: jacobi_oe_kernel, X held in registers (see its comment).
// l  > 128: the block form (jacobi_blk_*), block pairs of 16 + 16 columns in
//           registers, one launch per round of block pairs.
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "../../include/rsvd.h"

namespace rsvd {

constexpr int kJacobiRegMax = 128;
constexpr int kJacobiMaxSweeps = 60;

// Sum over the 8 lanes of each eighth of a wavefront (xor 1, xor 2, then
// lane i <-> 7 - i within each 8-lane half-row), result in all 8 lanes.
__device__ __forceinline__ double octet_sum(double x) {
    x += dpp_f64<dpp_quad_xor1>(x);
    x += dpp_f64<dpp_quad_xor2>(x);
    x += dpp_f64<dpp_half_mirror>(x);
    return x;
}

// Reciprocal and reciprocal square root: the hardware estimates refined by
// Newton steps (each squares the relative error), to full FP64 accuracy
// for normal arguments without the rescaling of the library forms.
__device__ __forceinline__ double rcp_newton(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double rsq_newton(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) y = fma(0.5 * y, fma(-(x * y), y, 1.0), y);
    return y;
}

// Tangent t of the Jacobi rotation for a column pair with squared norms a, b
// and inner product g: with d = b - a, e = 2g and r = (d^2 + e^2)^(1/2),
// t = sign(d) e / (|d| + r), the root of smaller magnitude of
// g t^2 + (b - a) t - g = 0, which makes the rotated pair orthogonal.  The
// form has no quotient that can overflow (the columns are scaled so that
// a, b <= 1, hence |d|, |e| <= 2) and no branch.  t = 0 (and `rot`
// untouched) when |g| <= tol sqrt(a b), the pair already orthogonal
// (tol2 = tol^2).
__device__ __forceinline__ double jacobi_tan(double a, double b, double g, int& rot, double tol2) {
    const bool r = g * g > tol2 * (a * b);
    rot |= (int)r;
    const double d = b - a, e = 2.0 * g;
    const double s2 = fma(d, d, e * e);
    const double t = (d >= 0.0 ? e : -e) * rcp_newton(fma(s2, rsq_newton(s2), fabs(d)));
    return r ? t : 0.0;
}

// A column of X as held by jacobi_oe_kernel: the true column is sc times the
// stored one; nr is its squared norm (tracked), isc = 1 / sc, id the
// original column index.
struct JColumn {
    double nr, sc, isc;
    int id;
};

// Rotation of the true pair (xi, xj) by tangent t (cosine c = (1 + t^2)^-1/2,
// sine s = c t): xi' = c xi - s xj, xj' = s xi + c xj.  With the cosine
// moved into the scales, the stored columns change by one FMA per element:
// yi' = yi - tr yj and yj' = yj + tir yi with tr = t sc_j / sc_i, tir = t sc_i
// / sc_j; the squared norms become a - t g and b + t g.
struct JRot {
    double tr, tir;
    JColumn ci, cj;
};
__device__ __forceinline__ JRot jacobi_rot(const JColumn& ci, const JColumn& cj, double g, double t) {
    const double u = fma(t, t, 1.0);
    const double c = rsq_newton(u), ic = u * c;
    JRot o;
    o.tr = t * (cj.sc * ci.isc);
    o.tir = t * (ci.sc * cj.isc);
    o.ci = {fma(-t, g, ci.nr), c * ci.sc, ic * ci.isc, ci.id};
    o.cj = {fma(t, g, cj.nr), c * cj.sc, ic * cj.isc, cj.id};
    return o;
}

template <int R>
__device__ __forceinline__ double partial_dot(const double (&xi)[R], const double (&xj)[R]) {
    double g0 = 0.0, g1 = 0.0;
#pragma unroll
    for (int k = 0; k < R; k += 2) {
        g0 = fma(xi[k], xj[k], g0);
        if (k + 1 < R) g1 = fma(xi[k + 1], xj[k + 1], g1);
    }
    return g0 + g1;
}

// Sorted singular values, U~ and M = U~ Sigma^-1 (L x L, zero padded) from
// the final columns; `nrm2` holds the squared norm of each original column
// (scaled by sc4), shared by the whole workgroup.
__device__ __forceinline__ void jacobi_rank(const double* nrm2, int* rank_of, int l, double sc4, double shift,
                                            double* sigma) {
    for (int c = threadIdx.x; c < l; c += blockDim.x) {
        const double sc = sqrt(fmax(nrm2[c] * sc4 - shift, 0.0));
        int rank = 0;
        for (int d = 0; d < l; ++d) {
            const double sd = sqrt(fmax(nrm2[d] * sc4 - shift, 0.0));
            rank += (sd > sc) || (sd == sc && d < c);   // stable descending order
        }
        rank_of[c] = rank;
        sigma[rank] = sc;
    }
}

// One-sided Jacobi for l <= 128 with X in registers.  Ordering: odd-even
// transposition.  Round r pairs the columns at positions (2i, 2i + 1) (r
// even) or (2i + 1, 2i + 2) (r odd), rotates each pair and swaps the two
// columns' positions; n (even) rounds make a sweep in which every pair of
// columns meets exactly once (the sequence is reversed, one adjacent swap
// per pair).
//
// A group of 8 lanes holds four consecutive positions 4g .. 4g + 3, lane e
// rows e + 8k (k < R, rows >= l zero); positions are padded to a multiple of
// 4 with zero columns, which never rotate.  Even rounds pair (4g, 4g + 1) and
// (4g + 2, 4g + 3), odd rounds (4g + 1, 4g + 2) inside the group and
// (4g + 3, 4g + 4) across neighbouring groups: group-local pairs need three
// DPP lane sums and no memory traffic, and only a group's first and last
// column go through LDS, once per two rounds.  Both groups of a cross pair
// compute its rotation (same inputs, same instructions, so both get the same
// rotation) and each keeps its own output column; the group-local middle
// pair is rotated while the neighbours' columns arrive.  The exchange
// alternates between two LDS buffers, so one barrier per two rounds orders
// it.  At l = 110: 28 groups on 4 wavefronts, one per SIMD.
//
// The odd round has no branches: a group at either end of the row pairs its
// end column with itself through LDS, with the inner product scaled by 0,
// which makes the rotation the identity (t = 0) and the update y' = 0 * y + y.
//
// Columns carry scales (JColumn), so a rotation costs one FMA per element
// and output; at the start of every sweep the scales are folded back in and
// the norms recomputed exactly.  X is first scaled by a power of two so
// that its largest column norm is about 1.  Sweeps stop when a whole sweep
// rotates nothing, or earlier when a test of all pairs at a sweep start
// finds none that would rotate: X^T X on FP64 MFMA (columns from the
// exchange buffer) against the same threshold as the rotations.  The test
// runs only after a sweep whose rotations all had |t| <= 2^-20, since with
// the quadratic convergence of the last sweeps nothing earlier can pass it;
// it saves the final sweep, which would rotate nothing.
// Independent problems of one launch (one workgroup each): problem b reads
// Rm + b * r and shift_p[b] and writes sigma + b * s, Ut + b * o, Mv + b * o.
struct JBatch {
    int64_t r, o;
    int s;
};

template <int R>
__global__ __launch_bounds__(256) void jacobi_oe_kernel(const double* __restrict__ Rm, int l, int L,
                                                        const double* __restrict__ shift_p,
                                                        double* __restrict__ sigma, double* __restrict__ Ut,
                                                        double* __restrict__ Mv, DevFlags* flags, int max_sweeps,
                                                        JBatch bs, double tol) {
    constexpr int LPP = 8, QMAX = kJacobiRegMax / 4;
    const double tol2 = tol * tol;
    Rm += blockIdx.x * bs.r;
    shift_p += blockIdx.x;
    sigma += blockIdx.x * bs.s;
    Ut += blockIdx.x * bs.o;
    Mv += blockIdx.x * bs.o;
    // [side][k][group][lane]: the four columns of each group for the test of
    // all pairs, or two exchange buffers of two sides (first column, last
    // column) for the rounds.
    constexpr int BUF = 4 * R * QMAX * LPP;
    static_assert(LPP * R <= kJacobiRegMax, "rows per column");
    __shared__ double xch[BUF];
    __shared__ JColumn xcol[4][QMAX];
    __shared__ double nrm2[kJacobiRegMax];
    __shared__ int rank_of[kJacobiRegMax];
    const int tid = threadIdx.x, gi = tid / LPP, e = tid % LPP;
    const int n4 = (l + 3) & ~3, G = n4 / 4;
    const bool active = gi < G;
    const bool hasR = gi < G - 1, hasL = active && gi > 0;
    auto xidx = [&](int side, int k, int g) { return ((side * R + k) * QMAX + g) * LPP + e; };

    double x[4][R];
    JColumn c[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int col = 4 * gi + s;
        c[s].id = col;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = e + LPP * k;
            x[s][k] = (active && col < l && r < l) ? Rm[(int64_t)col * L + r] : 0.0;
        }
    }
    for (int i = tid; i < kJacobiRegMax; i += blockDim.x) nrm2[i] = 0.0;
    __syncthreads();
    {
        double sq[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) sq[s] = octet_sum(partial_dot<R>(x[s], x[s]));
        if (active && e == 0) {
#pragma unroll
            for (int s = 0; s < 4; ++s) nrm2[4 * gi + s] = sq[s];
        }
    }
    __syncthreads();
    double mx = 0.0;
    for (int i = 0; i < n4; ++i) mx = fmax(mx, nrm2[i]);
    const int ex = mx > 0.0 ? ilogb(mx) / 2 : 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        c[s].sc = ldexp(1.0, -ex);
        c[s].isc = 1.0;
    }

    const int nwaves = (int)(blockDim.x / 64), wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    // An end group pairs its end column with itself: it reads back its own.
    const int sr = hasR ? 0 : 1, gr = hasR ? gi + 1 : gi;
    const int sl = hasL ? 1 : 0, gl = hasL ? gi - 1 : gi;
    bool converged = (l < 2), small = false;
    int sweeps_run = 0;
    int rot = 0, big = 0;
    // Rotation of the group-local pair at positions (p, p + 1); position p
    // takes the rotated second column.
    auto local = [&](double (&xa)[R], double (&xb)[R], JColumn& ca, JColumn& cb) {
        const double g = octet_sum(partial_dot<R>(xa, xb)) * (ca.sc * cb.sc);
        const double t = jacobi_tan(ca.nr, cb.nr, g, rot, tol2);
        big |= (int)(fabs(t) > 0x1.0p-20);
        const JRot o = jacobi_rot(ca, cb, g, t);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double yi = xa[k], yj = xb[k];
            xa[k] = fma(o.tir, yi, yj);
            xb[k] = fma(-o.tr, yj, yi);
        }
        ca = o.cj;
        cb = o.ci;
    };
    for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int k = 0; k < R; ++k) x[s][k] *= c[s].sc;
            c[s].sc = c[s].isc = 1.0;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) c[s].nr = octet_sum(partial_dot<R>(x[s], x[s]));
        if (small) {
            // Test of every pair of columns: G = X^T X, 16 x 16 tiles on and
            // above the diagonal, against |g| <= tol sqrt(a b) with the norms
            // of this sweep start.
#pragma unroll
            for (int s = 0; s < 4; ++s) {
#pragma unroll
                for (int k = 0; k < R; ++k) xch[xidx(s, k, gi)] = x[s][k];
            }
            if (e == 0) {
#pragma unroll
                for (int s = 0; s < 4; ++s) nrm2[4 * gi + s] = c[s].nr;
            }
            __syncthreads();
            const int ntc = (n4 + 15) / 16, ntiles = ntc * (ntc + 1) / 2;
            int bad = 0;
            for (int t = wave; t < ntiles; t += nwaves) {
                int a = 0, b = t;
                while (b >= ntc - a) { b -= ntc - a; ++a; }
                b += a;
                const int pa = 16 * a + li, pb = 16 * b + li;
                doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < LPP * R; kk += 4) {
                    const int row = kk + lk;       // row = e' + 8 k'
                    const int k = row / LPP, ee = row % LPP;
                    const double av = xch[(((pa & 3) * R + k) * QMAX + (pa >> 2)) * LPP + ee];
                    const double bv = xch[(((pb & 3) * R + k) * QMAX + (pb >> 2)) * LPP + ee];
                    acc = mfma16x16x4(av, bv, acc);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * a + acc_row<double>(lk, v), j = pb;
                    if (i < j && j < n4) bad |= (int)(acc[v] * acc[v] > tol2 * (nrm2[i] * nrm2[j]));
                }
            }
            if (!__syncthreads_or(bad)) {
                converged = true;
                break;
            }
        }
        ++sweeps_run;
        rot = 0;
        big = 0;
        for (int h = 0; h < 2 * G; ++h) {
            // even round: both pairs group-local
            local(x[0], x[1], c[0], c[1]);
            local(x[2], x[3], c[2], c[3]);
            // odd round: publish the end columns, rotate the middle pair, then
            // the two cross pairs
            const int b0 = 2 * (h & 1);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                xch[xidx(b0, k, gi)] = x[0][k];
                xch[xidx(b0 + 1, k, gi)] = x[3][k];
            }
            if (e == 0) {
                xcol[b0][gi] = c[0];
                xcol[b0 + 1][gi] = c[3];
            }
            __syncthreads();
            double yr[R], yl[R];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                yr[k] = xch[xidx(b0 + sr, k, gr)];
                yl[k] = xch[xidx(b0 + sl, k, gl)];
            }
            const JColumn cr = xcol[b0 + sr][gr], cl = xcol[b0 + sl][gl];
            local(x[1], x[2], c[1], c[2]);
            const double pr = partial_dot<R>(x[3], yr), pl = partial_dot<R>(yl, x[0]);
            const double gR = octet_sum(pr) * (hasR ? c[3].sc * cr.sc : 0.0);
            const double gL = octet_sum(pl) * (hasL ? cl.sc * c[0].sc : 0.0);
            const double tR = jacobi_tan(c[3].nr, cr.nr, gR, rot, tol2);
            const double tL = jacobi_tan(cl.nr, c[0].nr, gL, rot, tol2);
            big |= (int)(fmax(fabs(tR), fabs(tL)) > 0x1.0p-20);
            const JRot oR = jacobi_rot(c[3], cr, gR, tR);
            const JRot oL = jacobi_rot(cl, c[0], gL, tL);
            // Position 4g + 3 takes the rotated right neighbour, position 4g
            // the rotated left one (at an end: the column itself, t = 0).
#pragma unroll
            for (int k = 0; k < R; ++k) {
                x[3][k] = fma(oR.tir, x[3][k], yr[k]);
                x[0][k] = fma(-oL.tr, x[0][k], yl[k]);
            }
            c[3] = oR.cj;
            c[0] = oL.ci;
        }
        converged = !__syncthreads_or(rot);
        small = !__syncthreads_or(big);
    }
    if (!converged && tid == 0) atomicOr(&flags->info, RSVD_INFO_JACOBI_NOT_CONVERGED);
    if (tid == 0) atomicMax(&flags->jacobi_sweeps, sweeps_run);

#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int k = 0; k < R; ++k) x[s][k] *= c[s].sc;
    }
    __syncthreads();
    {
        double sq[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) sq[s] = octet_sum(partial_dot<R>(x[s], x[s]));
        if (active && e == 0) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if (c[s].id < l) nrm2[c[s].id] = sq[s];
        }
    }
    __syncthreads();
    const double shift = *shift_p, sc4 = ldexp(1.0, 2 * ex);
    jacobi_rank(nrm2, rank_of, l, sc4, shift, sigma);
    for (int idx = tid; idx < L * L; idx += blockDim.x) {
        Ut[idx] = 0.0;
        Mv[idx] = 0.0;
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cid = c[q].id;
            if (cid >= l) continue;
            const double nc = sqrt(nrm2[cid]);
            const double sv = sqrt(fmax(nrm2[cid] * sc4 - shift, 0.0));
            const double inv = nc > 0.0 ? 1.0 / nc : 0.0;
            const int col = rank_of[cid];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int r = e + LPP * k;
                if (r < l) {
                    const double u = nc > 0.0 ? x[q][k] * inv : (r == cid ? 1.0 : 0.0);
                    Ut[(int64_t)r * L + col] = u;
                    Mv[(int64_t)r * L + col] = sv > 0.0 ? u / sv : 0.0;
                }
            }
        }
    }
}

// Round-robin (circle method) schedule: with n2 (even) columns, round r pairs
// slot 0 with (n2 - 1, r) and slot s > 0 with ((r + s), (r - s)) mod (n2 - 1).
__device__ __forceinline__ void rr_pair(int r, int s, int n2, int& p1, int& p2) {
    const int m = n2 - 1;
    if (s == 0) { p1 = m; p2 = r; return; }
    p1 = r + s; if (p1 >= m) p1 -= m;
    p2 = r - s + m; if (p2 >= m) p2 -= m;
}

// ------------------------------------------------ block form, l > 128 --
// X = R^T (l x l) does not fit on one CU, and the single-workgroup form
// above streams all of X through that CU's cache every round.  This form
// splits the columns into blocks of 16 (a zero block is added when their
// number is odd) and orders the block pairs round-robin: a round is one
// launch in which every workgroup takes one pair of blocks, loads its 32
// columns into registers (16 lanes per column, rows e + 16 k), rotates them
// and writes them back.  The first round of a sweep runs one odd-even
// transposition sweep over the 32 columns (every pair of them meets once,
// the ordering of jacobi_oe_kernel), which covers the pairs inside every
// block; the later rounds meet only the cross pairs of their two blocks
// (jacobi_blk_cross_kernel).  The launches of a sweep together meet every
// pair of columns once; the kernel boundaries order the rounds, so no
// workgroup waits for another.  A word per
// sweep records whether any pair rotated; the launches of a sweep return at
// once when the previous sweep rotated nothing.  X is kept with column
// stride kMaxL; rows >= l are zero and stay zero.
constexpr int kBlkLpp = 16;
constexpr int kBlkGroups = 16;                 // 32 columns per workgroup

// X = 2^-ex R^T (zero padded), ex from the largest column norm; the sweep
// words cleared; 2^{2 ex} stored after the sweep words.
__global__ __launch_bounds__(1024) void jacobi_blk_prep_kernel(const double* __restrict__ R, int l, int L,
                                                               double* __restrict__ work) {
    __shared__ double red[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double* X = work;
    int* rotw = reinterpret_cast<int*>(work + (size_t)kMaxL * kMaxL);
    double mx = 0.0;
    for (int c = wid; c < l; c += 16) {           // wavefront per column
        double s2 = 0.0;
        for (int r = lane; r < l; r += 64) s2 = fma(R[(int64_t)c * L + r], R[(int64_t)c * L + r], s2);
        mx = fmax(mx, wave_sum(s2));
    }
    if (lane == 0) red[wid] = mx;
    __syncthreads();
    mx = 0.0;
    for (int w = 0; w < 16; ++w) mx = fmax(mx, red[w]);
    const int ex = mx > 0.0 ? ilogb(mx) / 2 : 0;
    const double sc = ldexp(1.0, -ex);
    for (int idx = tid; idx < kMaxL * kMaxL; idx += 1024) {
        const int c = idx / kMaxL, r = idx - c * kMaxL;
        X[idx] = (c < l && r < l) ? R[(int64_t)c * L + r] * sc : 0.0;
    }
    for (int i = tid; i < kJacobiBlockSweeps; i += 1024) rotw[i] = 0;
    if (tid == 0) work[(size_t)kMaxL * kMaxL + kJacobiBlockSweeps / 2 + 2] = ldexp(1.0, 2 * ex);
}

template <int R>
__global__ __launch_bounds__(kBlkLpp * kBlkGroups) void jacobi_blk_pair_kernel(double* __restrict__ work, int nb2,
                                                                                int round, int sweep, double tol) {
    constexpr int LPP = kBlkLpp, G = kBlkGroups;
    const double tol2 = tol * tol;
    __shared__ double xch[2 * R * G * LPP];          // [side][k][group][lane]
    __shared__ JColumn xcol[2][G];
    double* X = work;
    int* rotw = reinterpret_cast<int*>(work + (size_t)kMaxL * kMaxL);
    if (sweep > 0 && rotw[sweep - 1] == 0) return;   // the previous sweep rotated nothing
    const int tid = threadIdx.x, gi = tid / LPP, e = tid % LPP;
    auto xidx = [&](int side, int k, int g) { return ((side * R + k) * G + g) * LPP + e; };
    int p1, p2;
    rr_pair(round, blockIdx.x, nb2, p1, p2);
    const int b0 = min(p1, p2), b1 = max(p1, p2);
    auto colof = [&](int pos) { return pos < 16 ? 16 * b0 + pos : 16 * b1 + pos - 16; };
    double x0[R], x1[R];
    JColumn c0, c1;
    c0.id = colof(2 * gi);
    c1.id = colof(2 * gi + 1);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        x0[k] = X[(int64_t)c0.id * kMaxL + e + LPP * k];
        x1[k] = X[(int64_t)c1.id * kMaxL + e + LPP * k];
    }
    c0.sc = c1.sc = c0.isc = c1.isc = 1.0;
    c0.nr = quarter_sum(partial_dot<R>(x0, x0));
    c1.nr = quarter_sum(partial_dot<R>(x1, x1));
    const bool hasR = gi < G - 1, hasL = gi > 0;
    const int sr = hasR ? 0 : 1, gr = hasR ? gi + 1 : gi;
    const int sl = hasL ? 1 : 0, gl = hasL ? gi - 1 : gi;
    int rot = 0;
    for (int h = 0; h < G; ++h) {
        {   // even round: pair (2g, 2g + 1); position 2g takes the rotated second column
            const double g = quarter_sum(partial_dot<R>(x0, x1)) * (c0.sc * c1.sc);
            const double t = jacobi_tan(c0.nr, c1.nr, g, rot, tol2);
            const JRot o = jacobi_rot(c0, c1, g, t);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const double yi = x0[k], yj = x1[k];
                x0[k] = fma(o.tir, yi, yj);
                x1[k] = fma(-o.tr, yj, yi);
            }
            c0 = o.cj;
            c1 = o.ci;
        }
        // odd round: pairs (2g + 1, 2g + 2) across neighbouring groups (an end
        // group pairs with itself, t = 0)
#pragma unroll
        for (int k = 0; k < R; ++k) {
            xch[xidx(0, k, gi)] = x0[k];
            xch[xidx(1, k, gi)] = x1[k];
        }
        if (e == 0) {
            xcol[0][gi] = c0;
            xcol[1][gi] = c1;
        }
        __syncthreads();
        double yr[R], yl[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            yr[k] = xch[xidx(sr, k, gr)];
            yl[k] = xch[xidx(sl, k, gl)];
        }
        const JColumn cr = xcol[sr][gr], cl = xcol[sl][gl];
        __syncthreads();
        const double pr = partial_dot<R>(x1, yr), pl = partial_dot<R>(yl, x0);
        const double gR = hasR ? quarter_sum(pr) * (c1.sc * cr.sc) : 0.0;
        const double gL = hasL ? quarter_sum(pl) * (cl.sc * c0.sc) : 0.0;
        const double tR = jacobi_tan(c1.nr, cr.nr, gR, rot, tol2);
        const double tL = jacobi_tan(cl.nr, c0.nr, gL, rot, tol2);
        const JRot oR = jacobi_rot(c1, cr, gR, tR);
        const JRot oL = jacobi_rot(cl, c0, gL, tL);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            x1[k] = fma(oR.tir, x1[k], yr[k]);
            x0[k] = fma(-oL.tr, x0[k], yl[k]);
        }
        c1 = oR.cj;
        c0 = oL.ci;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        X[(int64_t)c0.id * kMaxL + e + LPP * k] = x0[k] * c0.sc;
        X[(int64_t)c1.id * kMaxL + e + LPP * k] = x1[k] * c1.sc;
    }
    if (__syncthreads_or(rot) && tid == 0) atomicOr(&rotw[sweep], 1);
}

// The later block rounds of a sweep: the block pair's 256 cross pairs (one
// column of each block) in 16 rounds instead of a full sweep over its 32
// columns.  Group g keeps column g of the first block and meets column
// (g + r) mod 16 of the second in round r; the second block's columns move
// one group down the ring through LDS after each round (two buffers, one
// barrier per round).  The pairs inside a block meet in the first block
// round of every sweep (jacobi_blk_pair_kernel, where each block takes part
// once), so every pair of columns still meets once per sweep.
template <int R>
__global__ __launch_bounds__(kBlkLpp * kBlkGroups) void jacobi_blk_cross_kernel(double* __restrict__ work, int nb2,
                                                                                 int round, int sweep, double tol) {
    constexpr int LPP = kBlkLpp, G = kBlkGroups;
    const double tol2 = tol * tol;
    __shared__ double xch[2 * R * G * LPP];          // [buffer][k][group][lane]
    __shared__ JColumn xcol[2][G];
    double* X = work;
    int* rotw = reinterpret_cast<int*>(work + (size_t)kMaxL * kMaxL);
    if (sweep > 0 && rotw[sweep - 1] == 0) return;   // the previous sweep rotated nothing
    const int tid = threadIdx.x, gi = tid / LPP, e = tid % LPP;
    auto xidx = [&](int buf, int k, int g) { return ((buf * R + k) * G + g) * LPP + e; };
    int p1, p2;
    rr_pair(round, blockIdx.x, nb2, p1, p2);
    const int b0 = min(p1, p2), b1 = max(p1, p2);
    double x0[R], x1[R];                             // column gi of block b0; the visiting column of b1
    JColumn c0, c1;
    c0.id = 16 * b0 + gi;
    c1.id = 16 * b1 + gi;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        x0[k] = X[(int64_t)c0.id * kMaxL + e + LPP * k];
        x1[k] = X[(int64_t)c1.id * kMaxL + e + LPP * k];
    }
    c0.sc = c1.sc = c0.isc = c1.isc = 1.0;
    c0.nr = quarter_sum(partial_dot<R>(x0, x0));
    c1.nr = quarter_sum(partial_dot<R>(x1, x1));
    const int gn = (gi + 1) % G;                     // the group whose column arrives next
    int rot = 0;
    for (int r = 0; r < G; ++r) {
        const double g = quarter_sum(partial_dot<R>(x0, x1)) * (c0.sc * c1.sc);
        const double t = jacobi_tan(c0.nr, c1.nr, g, rot, tol2);
        const JRot o = jacobi_rot(c0, c1, g, t);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double yi = x0[k], yj = x1[k];
            x0[k] = fma(-o.tr, yj, yi);
            x1[k] = fma(o.tir, yi, yj);
        }
        c0 = o.ci;
        c1 = o.cj;
        if (r + 1 < G) {
            const int buf = r & 1;
#pragma unroll
            for (int k = 0; k < R; ++k) xch[xidx(buf, k, gi)] = x1[k];
            if (e == 0) xcol[buf][gi] = c1;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < R; ++k) x1[k] = xch[xidx(buf, k, gn)];
            c1 = xcol[buf][gn];
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        X[(int64_t)c0.id * kMaxL + e + LPP * k] = x0[k] * c0.sc;
        X[(int64_t)c1.id * kMaxL + e + LPP * k] = x1[k] * c1.sc;
    }
    if (__syncthreads_or(rot) && tid == 0) atomicOr(&rotw[sweep], 1);
}

// Column norms of the final X, sorted singular values, U~ and M = U~ Sigma^-1
// (as at the end of the other forms); the sweep cap flag.
__global__ __launch_bounds__(512) void jacobi_blk_finish_kernel(const double* __restrict__ work, int l, int L,
                                                                const double* __restrict__ shift_p,
                                                                double* __restrict__ sigma, double* __restrict__ Ut,
                                                                double* __restrict__ Mv, DevFlags* flags,
                                                                int sweeps) {
    __shared__ double nrm2[kMaxL];
    __shared__ int rank_of[kMaxL];
    const double* X = work;
    const int* rotw = reinterpret_cast<const int*>(work + (size_t)kMaxL * kMaxL);
    const double sc4 = work[(size_t)kMaxL * kMaxL + kJacobiBlockSweeps / 2 + 2];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) {
        if (rotw[sweeps - 1] != 0) atomicOr(&flags->info, RSVD_INFO_JACOBI_NOT_CONVERGED);
        int run = 0;                  // sweeps until (and with) the first one that rotated nothing
        while (run < sweeps && rotw[run] != 0) ++run;
        atomicMax(&flags->jacobi_sweeps, min(run + 1, sweeps));
    }
    for (int c = wid; c < l; c += 8) {
        double s2 = 0.0;
        for (int r = lane; r < l; r += 64) s2 = fma(X[(int64_t)c * kMaxL + r], X[(int64_t)c * kMaxL + r], s2);
        s2 = wave_sum(s2);
        if (lane == 0) nrm2[c] = s2;
    }
    __syncthreads();
    const double shift = *shift_p;
    jacobi_rank(nrm2, rank_of, l, sc4, shift, sigma);
    __syncthreads();
    for (int idx = tid; idx < L * L; idx += 512) {
        Ut[idx] = 0.0;
        Mv[idx] = 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < l * l; idx += 512) {
        const int c = idx / l, row = idx - c * l;
        const double nc = sqrt(nrm2[c]);
        const double sv = sqrt(fmax(nrm2[c] * sc4 - shift, 0.0));
        const double u = nc > 0.0 ? X[(int64_t)c * kMaxL + row] / nc : (row == c ? 1.0 : 0.0);
        const int col = rank_of[c];
        Ut[(int64_t)row * L + col] = u;
        Mv[(int64_t)row * L + col] = sv > 0.0 ? u / sv : 0.0;
    }
}

template <int R>
static void launch_jacobi_blk(const double* Rm, int l, int L, const double* shift, double* sigma, double* Ut,
                              double* Mv, DevFlags* flags, double* work, hipStream_t s, int sweeps, double tol) {
    const int nb = (l + 15) / 16, nb2 = nb + (nb & 1);
    hipLaunchKernelGGL(jacobi_blk_prep_kernel, dim3(1), dim3(1024), 0, s, Rm, l, L, work);
    for (int sweep = 0; sweep < sweeps; ++sweep) {
        hipLaunchKernelGGL(jacobi_blk_pair_kernel<R>, dim3(nb2 / 2), dim3(kBlkLpp * kBlkGroups), 0, s, work, nb2, 0,
                           sweep, tol);
        for (int r = 1; r < nb2 - 1; ++r)
            hipLaunchKernelGGL(jacobi_blk_cross_kernel<R>, dim3(nb2 / 2), dim3(kBlkLpp * kBlkGroups), 0, s, work,
                               nb2, r, sweep, tol);
    }
    hipLaunchKernelGGL(jacobi_blk_finish_kernel, dim3(1), dim3(512), 0, s, work, l, L, shift, sigma, Ut, Mv, flags,
                       sweeps);
}

template <int R>
static void launch_jacobi_oe(const double* Rm, int l, int L, const double* shift, double* sigma, double* Ut,
                             double* Mv, DevFlags* flags, hipStream_t s, int sweeps, int batch, JBatch bs,
                             double tol) {
    const int groups = ((l + 3) & ~3) / 4;
    const int threads = (int)round_up(groups * 8, kWave);
    hipLaunchKernelGGL(jacobi_oe_kernel<R>, dim3(batch), dim3(threads), 0, s, Rm, l, L, shift, sigma, Ut, Mv, flags,
                       sweeps, bs, tol);
}

hipError_t launch_jacobi(const double* R, int l, int L, const double* shift, double* sigma, double* Ut, double* Mv,
                         DevFlags* flags, double* work, double tol, hipStream_t s, int max_sweeps, int batch) {
    if (l < 1 || l > kMaxL || L < l || max_sweeps < 0 || batch < 1 || !(tol > 0.0 && tol < 1.0))
        return hipErrorInvalidValue;
    if (batch > 1 && l > kJacobiRegMax) return hipErrorInvalidValue;
    const JBatch bs{(int64_t)L * L, (int64_t)L * L, L};
    const int oe_sweeps = max_sweeps ? max_sweeps : kJacobiMaxSweeps;
    const int blk_sweeps = max_sweeps ? std::min(max_sweeps, kJacobiBlockSweeps) : kJacobiBlockSweeps;
    if (l <= kJacobiRegMax) {
        // rows per lane and column: 2 ceil(l / 16), so 8 lanes cover ceil(l / 16) * 16 >= l rows
        switch ((l + 15) / 16) {
            case 1: launch_jacobi_oe<2>(R, l, L, shift, sigma, Ut, Mv, flags, s, oe_sweeps, batch, bs, tol); break;
            case 2: launch_jacobi_oe<4>(R, l, L, shift, sigma, Ut, Mv, flags, s, oe_sweeps, batch, bs, tol); break;
            case 3: launch_jacobi_oe<6>(R, l, L, shift, sigma, Ut, Mv, flags, s, oe_sweeps, batch, bs, tol); break;
            case 4: launch_jacobi_oe<8>(R, l, L, shift, sigma, Ut, Mv, flags, s, oe_sweeps, batch, bs, tol); break;
            case 5: launch_jacobi_oe<10>(R, l, L, shift, sigma, Ut, Mv, flags, s, oe_sweeps, batch, bs, tol); break;
            case 6: launch_jacobi_oe<12>(R, l, L, shift, sigma, Ut, Mv, flags, s, oe_sweeps, batch, bs, tol); break;
            case 7: launch_jacobi_oe<14>(R, l, L, shift, sigma, Ut, Mv, flags, s, oe_sweeps, batch, bs, tol); break;
            default: launch_jacobi_oe<16>(R, l, L, shift, sigma, Ut, Mv, flags, s, oe_sweeps, batch, bs, tol); break;
        }
    } else {
        // rows per lane and column: ceil(l / 16), 16 lanes per column pair
        switch ((l + 15) / 16) {
            case 9: launch_jacobi_blk<9>(R, l, L, shift, sigma, Ut, Mv, flags, work, s, blk_sweeps, tol); break;
            case 10: launch_jacobi_blk<10>(R, l, L, shift, sigma, Ut, Mv, flags, work, s, blk_sweeps, tol); break;
            case 11: launch_jacobi_blk<11>(R, l, L, shift, sigma, Ut, Mv, flags, work, s, blk_sweeps, tol); break;
            case 12: launch_jacobi_blk<12>(R, l, L, shift, sigma, Ut, Mv, flags, work, s, blk_sweeps, tol); break;
            case 13: launch_jacobi_blk<13>(R, l, L, shift, sigma, Ut, Mv, flags, work, s, blk_sweeps, tol); break;
            case 14: launch_jacobi_blk<14>(R, l, L, shift, sigma, Ut, Mv, flags, work, s, blk_sweeps, tol); break;
            case 15: launch_jacobi_blk<15>(R, l, L, shift, sigma, Ut, Mv, flags, work, s, blk_sweeps, tol); break;
            case 16: launch_jacobi_blk<16>(R, l, L, shift, sigma, Ut, Mv, flags, work, s, blk_sweeps, tol); break;
            case 17: launch_jacobi_blk<17>(R, l, L, shift, sigma, Ut, Mv, flags, work, s, blk_sweeps, tol); break;
            default: launch_jacobi_blk<18>(R, l, L, shift, sigma, Ut, Mv, flags, work, s, blk_sweeps, tol); break;
        }
    }
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

__global__ void export_info_kernel(const DevFlags* flags, int* info, int* sweeps) {
    *info = flags->info;
    if (sweeps) *sweeps = flags->jacobi_sweeps;
}

hipError_t launch_export_info(const DevFlags* flags, int* info, hipStream_t s, int* sweeps) {
    hipLaunchKernelGGL(export_info_kernel, dim3(1), dim3(1), 0, s, flags, info, sweeps);
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

// Wide form: M = [-Q^T W; I_b] ((L + B) x B, ld B) from the Gram partials of
// [Q | W] (rows x (L + B), L and B multiples of 16); columns c >= b of M are
// zero.
__global__ __launch_bounds__(256) void proj_coef_w_kernel(const double* __restrict__ part, int nchunks, int L, int B,
                                                          int b, double* __restrict__ M) {
    const int nt = (L + B) / 16, npairs = nt * (nt + 1) / 2;
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < (L + B) * B; idx += 256 * gridDim.x) {
        const int a = idx / B, c = idx % B;
        double v = 0.0;
        if (c < b) {
            if (a < L) {
                const int ta = a >> 4, tb = (L + c) >> 4;
                const int pr = ta * nt - ta * (ta - 1) / 2 + (tb - ta);   // row-major upper-triangle index
                const int e = (a & 15) * 16 + ((L + c) & 15);
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

hipError_t launch_proj_coef_w(const double* partials, int64_t rows, int L, int B, int b, double* M, hipStream_t s) {
    if (L % 16 || B % 16 || L + B > kMaxL || b > B) return hipErrorInvalidValue;
    hipLaunchKernelGGL(proj_coef_w_kernel, dim3((unsigned)ceil_div((L + B) * B, 256)), dim3(256), 0, s, partials,
                       gram_chunks(rows), L, B, b, M);
    return hipGetLastError();
}

// sines[j] = min(1, sigma[k - 1 - j]): the singular values of the projection
// residual, ascending.
__global__ void sines_kernel(const double* sigma, int k, double* sines) {
    for (int j = threadIdx.x; j < k; j += blockDim.x) sines[j] = fmin(1.0, sigma[k - 1 - j]);
}

hipError_t launch_sines(const double* sigma, int k, double* sines, hipStream_t s) {
    hipLaunchKernelGGL(sines_kernel, dim3(1), dim3(256), 0, s, sigma, k, sines);
    return hipGetLastError();
}

// Adaptive range finder, per block: est = factor * max_i ||y_i|| (column
// norms from the diagonal of the Gram partials of the block, B wide) and
// keep = #{sigma_i > thr} over the block's b sorted singular values.
// out[0] = est, out[1] = keep.
__global__ __launch_bounds__(64) void adaptive_stats_kernel(const double* __restrict__ part, int nchunks, int B, int b,
                                                            const double* __restrict__ sigma, double factor, double thr,
                                                            double* out) {
    const int nt = B / 16, npairs = nt * (nt + 1) / 2;
    double mx = 0.0;
    int keep = 0;
    for (int c = threadIdx.x; c < b; c += 64) {
        const int t = c >> 4;
        const int pr = t * nt - t * (t - 1) / 2;                   // diagonal tile (t, t)
        const int e = (c & 15) * 16 + (c & 15);
        double sq = 0.0;
        for (int ch = 0; ch < nchunks; ++ch) sq += part[((size_t)ch * npairs + pr) * 256 + e];
        mx = fmax(mx, sqrt(fmax(sq, 0.0)));
        keep += sigma[c] > thr ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o));
        keep += __shfl_xor(keep, o);
    }
    if (threadIdx.x == 0) {
        out[0] = factor * mx;
        out[1] = (double)keep;
    }
}

hipError_t launch_adaptive_stats(const double* partials, int64_t rows, int B, int b, const double* sigma,
                                 double factor, double thr, double* out, hipStream_t s) {
    hipLaunchKernelGGL(adaptive_stats_kernel, dim3(1), dim3(64), 0, s, partials, gram_chunks(rows), B, b, sigma, factor,
                       thr, out);
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
