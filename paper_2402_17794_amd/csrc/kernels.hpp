// Internal launcher interface between the host driver and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

// Largest padded width L = 16 * LT supported by the product kernels.
constexpr int kMaxLT = 18;
constexpr int kMaxL = 16 * kMaxLT;
constexpr int kMaxSplits = 16;     // split-K slices of a product with A

// Status flags kept in device memory for one orthonormalisation / solve.
struct DevFlags {
    int orth_fail;      // CholeskyQR breakdown in the current orth -> Householder
    int info;           // RSVD_INFO_* bits accumulated over the solve
    int pass2_off;      // the second CholeskyQR pass of the current orth does not run
    int fb_count;       // grid barrier of the Householder fallback: arrivals (0 between barriers)
    int fb_gen;         // and its generation
    int jacobi_sweeps;  // sweeps the small SVD's Jacobi iteration ran (the last one rotates nothing)
    int pad[58];
};

// ---- skinny products with A (gemm.hip) ----
struct GemmArgs {
    const void* A; int64_t lda;
    int trans;                 // 0: Y = A X (M = rows of A, K = cols); 1: Y = A^T X
    int64_t M, K;              // output rows, reduction length
    const void* X; int64_t ldx;  // K x ncols; NULL with trans = 0 -> Omega(seed)
    uint64_t seed;
    int ncols;                 // valid columns of X / Y (<= kMaxL)
    int wcols;                 // columns of Y to write (ncols or L)
    void* Y; int64_t ldy;
    void* partials;            // splits * M * L elements (splits > 1)
    int splits;
    int omega_kind;            // X == NULL: kOmegaGaussian (default) or kOmegaSrft
    const int* srft_cols;      // kOmegaSrft: the ncols sampled DCT columns (device)
    uint32_t omega_stream;     // kOmegaGaussian: Philox stream id (0 = the solve's test matrix)
    int64_t omega_col0;        // kOmegaGaussian: column j of the product uses test-matrix column col0 + j
};
constexpr int kOmegaGaussian = 0, kOmegaSrft = 1;
size_t gemm_partials_elems(int dtype, int64_t M, int64_t K, int ncols, int* splits_out);
int gemm_row_tiles(int dtype, int64_t M, int ncols);
// product_done (optional) is recorded on s right after the product kernel,
// before the split-K reduction, so that it times the product alone.
hipError_t launch_gemm(int dtype, GemmArgs a, hipStream_t s, hipEvent_t product_done = nullptr);

// Y (ldy, first wcols columns) = sum of the `splits` FP32 slices of M x L
// partial products, in slice order.
hipError_t launch_splitk_reduce_f32(const float* partials, int64_t M, int L, int splits, float* Y, int64_t ldy,
                                    int wcols, hipStream_t s);

// ---- two-sided sketch of the single-pass Algorithm 6 (gemm.hip) ----
// Y_c = A Omega_c (M x l, Philox stream stream_c over the K rows of Omega_c)
// and Y_r = A^T Omega_r (K x l, stream stream_r over the M rows of Omega_r)
// from one read of A (M x K, FP32 or FP64).  l <= kMaxDualL.
constexpr int kMaxDualL = 144;
struct DualArgs {
    const void* A; int64_t lda;
    int64_t M, K;
    uint64_t seed;
    int ncols;                 // l
    int wcols;                 // columns of Y_c / Y_r to write (l or L)
    uint32_t stream_c, stream_r;
    void* Yc; int64_t ldyc;    // M x wcols
    void* part_c;              // splits * M * L (splits > 1)
    int splits;
    void* part_r;              // dual_row_tiles * K * L: per row tile partials of Y_r
    void* omega_c_out; int64_t ldoc;   // nullable: Omega_c (K x L, zero past l)
    void* omega_r_out; int64_t ldor;   // nullable: Omega_r (M x L, zero past l)
};
int dual_row_tiles(int dtype, int64_t M);
int dual_splits(int dtype, int64_t M, int64_t K);
// Launches the product kernel (product_done, optional, is recorded right
// after it), the split-K reduction of Y_c and the row-tile reduction of Y_r
// into Yr (K x wcols, ld ldyr).
hipError_t launch_dual_sketch(int dtype, DualArgs a, void* Yr, int64_t ldyr, hipStream_t s,
                              hipEvent_t product_done = nullptr);

// ---- Stage 2 of the single-pass algorithms (single_pass.hip) ----
// out (LX x LZ FP64, ld ldo) = X^T Z for X rows x LX, Z rows x LZ (dtype,
// LX, LZ multiples of 16); partials: cross_partials_elems doubles.
size_t cross_partials_elems(int64_t rows, int LX, int LZ);
hipError_t launch_cross(int dtype, const void* X, int64_t ldx, const void* Z, int64_t ldz, int64_t rows, int LX,
                        int LZ, double* partials, double* out, int ldo, hipStream_t s);
// C (Mw x Nw, ldc) = op(A) op(B) on the leading M x N block, zero elsewhere;
// with dr, dc: each element divided by dr[i]^2 + dc[j]^2.
hipError_t launch_small_gemm(int M, int N, int K, const double* A, int lda, int ta, const double* B, int ldb, int tb,
                             double* C, int ldc, int Mw, int Nw, hipStream_t s, const double* dr = nullptr,
                             const double* dc = nullptr);
// X (l x l, ldx) with W^T X = Z^T (Gauss-Jordan, partial pivoting), l <= 128.
hipError_t launch_gj_solve(const double* Wt, const double* Zt, int ld, int l, double* X, int ldx, DevFlags* flags,
                           hipStream_t s);
// Symmetric part of X shifted by *shift = 2 ||sym(X)||_F, as Gram partials.
hipError_t launch_sym_pack(const double* X, int ldx, int l, int L, double* partials, double* shift, hipStream_t s);
// Eigenvalues sigma^2 - shift, the k of largest magnitude with their vectors.
hipError_t launch_eig_finish(const double* sigma, const double* Ut, int l, int L, const double* shift, int k,
                             double* lam_out, double* Wu, int ldw, hipStream_t s);

// ---- products with a low-precision A (gemm_lp.hip) ----
constexpr int kFmtBf16 = 2, kFmtFp8 = 3;           // RSVD_BF16, RSVD_FP8_E4M3
struct LpGemmArgs {
    const void* A; int64_t lda;     // BF16 or FP8 A, ld in elements (a multiple of 16 bytes), 16-byte aligned
    const float* col_scale;         // FP8: the column scales of A, else NULL
    int trans;                      // 0: Y = A X (M = rows, K = cols); 1: Y = A^T X
    int64_t M, K;
    const void* Xt; int64_t ldt;    // prepared operand (L x ldt, k-contiguous); NULL with trans = 0 -> Omega
    const float* xscale;            // FP8: column scales of the operand (ncols), else NULL
    const float* omega_scale;       // FP8 sketch: device pointer to max_j col_scale_j
    uint64_t seed;
    int ncols, wcols;
    float* Y; int64_t ldy;
    float* partials;                // splits * M * L floats (splits > 1)
    int splits;
};
// FP32 A (rows x cols, lda) -> BF16 or column-scaled FP8 (col_scale: cols floats).
hipError_t launch_quantize(int fmt, const float* A, int64_t rows, int64_t cols, int64_t lda, void* Q, int64_t ldq,
                           float* col_scale, hipStream_t s);
// X (K x ncols FP32, ldx) -> Xt (L x ldt, k-contiguous, zero padded; ldt a
// multiple of 64 >= K) in the format of A; FP8 also writes the column
// scales tscale (ncols) and uses amax_tmp (L words).  row_scale (FP8, K
// floats, nullable) multiplies the rows of X first.
hipError_t launch_lp_operand(int fmt, const float* X, int64_t K, int ncols, int64_t ldx, const float* row_scale,
                             void* Xt, int64_t ldt, int L, float* tscale, unsigned* amax_tmp, hipStream_t s);
hipError_t launch_vec_max(const float* v, int64_t n, float* out, hipStream_t s);
size_t lp_partials_elems(int64_t M, int64_t K, int ncols, int* splits_out);
hipError_t launch_lp_gemm(int fmt, LpGemmArgs a, hipStream_t s, hipEvent_t product_done = nullptr);

// ---- Gram, Cholesky, apply, Householder (orth.hip) ----
// Chunk partials of G = Y^T Y (FP64) for Y rows x L (dtype, zero padding):
// gram_partials_elems doubles, consumed by launch_chol with the same rows.
int gram_chunks(int64_t rows);
size_t gram_partials_elems(int64_t rows, int L);
int gram_pairs(int L);
// skip (nullable): the kernel returns at once when *skip != 0.
hipError_t launch_gram(int dtype, const void* Y, int64_t ldy, int64_t rows, int L, double* partials,
                       const int* skip, hipStream_t s);

// Sum the Gram partials and factor G = R^T R, forming R^{-1} too (single
// workgroup); R, Rinv: L x L, zero outside the leading l x l block.
// mode 0 (orth pass 1): on breakdown set flags->orth_fail = 1 (else 0);
//                       flags->pass2_off = 1 on breakdown, or when
//                       skip_tau > 0 and rows 2^-53 sum_ij G_ii Rinv_ij^2 <=
//                       skip_tau (the first pass is already orthonormal to
//                       below skip_tau), else 0.
// mode 1 (orth pass 2): return at once if pass2_off; first-order factor when
//                       max |G - I| <= tau; on breakdown set orth_fail = 1
//                       and pass2_off = 1.
// mode 2 (small SVD): on breakdown retry with a diagonal shift, report it in
//                     info and store the shift in *shift_out.
// report_breakdown (modes 0, 1): also set RSVD_INFO_ORTH_BREAKDOWN on breakdown.
// work: L*L doubles of device scratch (used when l is too large for LDS).
hipError_t launch_chol(const double* partials, int64_t rows, int l, int L, double* R, double* Rinv,
                       DevFlags* flags, int mode, double* shift_out, double* work, double tau, hipStream_t s,
                       double skip_tau = 0.0, int report_breakdown = 0);

// out[rows x ncols_out] = in[rows x L] * M[L x ncols_out] with FP64 accumulation.
// transpose_out: write out^T (ncols_out x rows, ld = ldo).  colscale (nullable):
// multiply output column c by colscale[c].  skip (nullable): return at once
// if *skip != 0.  argmax (nullable, with transpose_out): per-block
// index/value of the largest |entry| of each output column.
// upper: M is upper triangular (its zero blocks are skipped).
// out may be in (same ld, no transpose): every workgroup reads all of its
// rows before it writes them.
hipError_t launch_apply(int dtype, const void* in, int64_t ldi, int64_t rows, int L, const double* M, int ldm,
                        int ncols_out, void* out, int64_t ldo, int transpose_out, const double* colscale,
                        const int* skip, double* argmax_val, int* argmax_idx, int upper,
                        hipStream_t s);
int apply_blocks(int64_t rows);

// Householder QR fallback (TSQR tree over up to 64 workgroups); runs only if
// flags->orth_fail (or `force`).  H, Qw: rows * L doubles each; up:
// householder_scratch_doubles(rows, L) doubles.  Sets RSVD_INFO_QR_FALLBACK.
size_t householder_scratch_doubles(int64_t rows, int L);
hipError_t launch_householder(int dtype, const void* Y, int64_t ldy, int64_t rows, int l, int L, void* Q,
                              int64_t ldq, double* H, double* Qw, double* up, DevFlags* flags, int force,
                              hipStream_t s);

// ---- small SVD and finishing (svd.hip) ----
// One-sided Jacobi on X = R^T (l x l, from the Cholesky factor of B B^T).
// Outputs sigma (sorted descending, shift removed), Ut (L x L, column c =
// left singular vector c of B, sorted), Mv (L x L: Ut * diag(1/sigma)),
// work: kJacobiWorkDoubles doubles of device scratch (used when l > 128).
constexpr int kJacobiBlockSweeps = 30;                   // sweep cap of the l > 128 form
constexpr size_t kJacobiWorkDoubles = (size_t)kMaxL * kMaxL + kJacobiBlockSweeps + 8;
// max_sweeps: sweep cap (0 = the default of the form); reaching it sets
// RSVD_INFO_JACOBI_NOT_CONVERGED.  flags->jacobi_sweeps receives the largest
// sweep count of the solve's small SVDs.  batch (l <= 128 only): that many
// independent problems of the same l in one launch, one workgroup each,
// problem b at R + b L^2, shift + b, sigma + b L, Ut + b L^2, Mv + b L^2.
// tol: rotation threshold, a pair rotates while |x_i . x_j| > tol |x_i| |x_j|
// (0 < tol < 1).
hipError_t launch_jacobi(const double* R, int l, int L, const double* shift, double* sigma, double* Ut,
                         double* Mv, DevFlags* flags, double* work, double tol, hipStream_t s, int max_sweeps = 0,
                         int batch = 1);

// Reduce the per-block argmax partials of the V columns, choose signs,
// write S (r values) and sign[c].
hipError_t launch_signs(const double* argmax_val, const int* argmax_idx, int nblocks, int r,
                        const double* sigma, double* S_out, double* sign, hipStream_t s);

// Scale the rows of a (rows x cols, ld) matrix of dtype by sign[row].
hipError_t launch_scale_rows(int dtype, void* X, int64_t ld, int rows, int64_t cols, const double* sign,
                             hipStream_t s);

// dst (rows x dcols, ldd) = src (rows x cols, lds) padded with zero columns.
hipError_t launch_copy2d(int dtype, const void* src, int64_t lds, int64_t rows, int cols, void* dst, int64_t ldd,
                         int dcols, hipStream_t s);

// Zero `count` ints and the flags block.
hipError_t launch_init(int* counters, int count, DevFlags* flags, hipStream_t s);
// Write the flags' info word to the caller's info (an assignment: the
// caller's word needs no initialisation).
// sweeps (nullable): also the Jacobi sweep count of the small SVD.
hipError_t launch_export_info(const DevFlags* flags, int* info, hipStream_t s, int* sweeps = nullptr);

// SRFT test matrix: the l sampled columns of the DCT-II (Floyd's algorithm
// on Philox stream 4), one wavefront; and the matrix materialised.
hipError_t launch_srft_columns(uint64_t seed, int64_t n, int l, int* cols, hipStream_t s);
hipError_t launch_srft_omega(int dtype, uint64_t seed, int64_t n, int l, const int* cols, void* out, int64_t ld,
                             hipStream_t s);
// Omega materialised / raw Philox words (test entry points).
hipError_t launch_omega(int dtype, uint64_t seed, uint32_t stream, int64_t n, int64_t l, void* out, int64_t ld,
                        hipStream_t s);
hipError_t launch_philox_words(uint64_t seed, uint32_t stream, const uint32_t* ctr, int64_t count, uint32_t* out,
                               hipStream_t s);

// ||A - Q B||_F with B^T = Bt (n x L): tile partials (FP64 accumulation of
// squares) and a fixed-order final sum; out[0] = 0, out[1] = the norm.
hipError_t launch_residual_fro(int dtype, const void* A, int64_t lda, int64_t m, int64_t n, const void* Q,
                               const void* Bt, int l, int L, double* partial, double* out, hipStream_t s);
size_t residual_partials(int64_t m, int64_t n);

// Spectral-norm estimator of A - Q Q^T A: M = [-Q^T W; I_b] ((L + 16) x 16,
// FP64) from the Gram partials of [Q | W] (rows x (L + 16)).
hipError_t launch_proj_coef(const double* partials, int64_t rows, int L, int b, double* M, hipStream_t s);
// Wide form of launch_proj_coef: M = [-Q^T W; I_b] ((L + B) x B, ld B) from
// the Gram partials of [Q | W] (rows x (L + B)); columns >= b zero.
hipError_t launch_proj_coef_w(const double* partials, int64_t rows, int L, int B, int b, double* M, hipStream_t s);
// sines[j] = min(1, sigma[k-1-j]) (ascending).
hipError_t launch_sines(const double* sigma, int k, double* sines, hipStream_t s);
// Adaptive range finder block statistics: out[0] = factor * largest column
// norm of the block (from the diagonal of its Gram partials, B wide),
// out[1] = number of the b sorted sigma above thr.
hipError_t launch_adaptive_stats(const double* partials, int64_t rows, int B, int b, const double* sigma,
                                 double factor, double thr, double* out, hipStream_t s);
// out[0] = sigma[0]; out[1] = 0 unless the Frobenius norm was requested.
hipError_t launch_residual_spec_final(const double* sigma, double* out, int fro_requested, hipStream_t s);

}  // namespace rsvd
