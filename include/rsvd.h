/*
 * rsvd.h - C ABI of the MI355X (gfx950) randomized SVD library (librsvd.so).
 *
 * The library computes the randomized SVD of Algorithm 4 of the thesis
 * (Chapter 3, Section 3.3, "accuracy enhanced randomized SVD with
 * orthonormalization"): for an m x n matrix A, target rank k, oversampling p
 * and power exponent q, with l = min(k + p, min(m, n)):
 *
 *   Omega  = n x l standard Gaussian test matrix          (step 1)
 *   Y      = A Omega,  Q = orth(Y)                          (steps 2-3)
 *   q times: W = orth(A^T Q),  Q = orth(A W)               (steps 4-5)
 *   B      = Q^T A,  B = U~ Sigma V^T,  U = Q U~            (steps 6-8)
 *
 * truncated to the top k singular triplets (Section 3.1, after Algorithm 2).
 * Algorithm 2 (Section 3.1) is the case q = 0.  The error measure
 * ||A - Q Q^T A|| of Theorems 2, 3 and 6 is available as an option.
 *
 * Conventions
 *  - Every matrix is dense, real and ROW-MAJOR with a leading dimension `ld`
 *    (elements between the starts of consecutive rows, ld >= cols).
 *  - All matrix and vector arguments are DEVICE pointers on the handle's
 *    device unless stated otherwise.  The caller owns every buffer; the
 *    library never frees caller memory and keeps no pointer after a call
 *    returns (asynchronous work enqueued on `stream` still uses them).
 *  - Work is enqueued asynchronously on the caller's `stream`
 *    (a hipStream_t passed as void*; NULL is the null stream).  Argument
 *    errors are detected on the host before anything is enqueued and
 *    returned synchronously.  Numerical conditions are reported in the
 *    device `info` word (bit flags below), readable after the stream is
 *    synchronised.
 *  - A handle is not thread-safe; use one per host thread.
 *  - Omega is never stored: it is generated inside the sketch kernel from
 *    (seed, row, column) by Philox4x32-10 and the Box-Muller transform
 *    (see rsvd_omega for the exact element definition), so a solve is a
 *    pure function of (A, k, p, q, seed).
 */
#ifndef RSVD_H
#define RSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSVD_OK = 0,
    RSVD_ERR_INVALID_ARG = 1,      /* bad pointer, size, leading dimension or parameter */
    RSVD_ERR_UNSUPPORTED = 2,      /* valid request this build does not implement */
    RSVD_ERR_NO_MEMORY = 3,        /* a host or device allocation failed */
    RSVD_ERR_WORKSPACE_TOO_SMALL = 4,
    RSVD_ERR_DEVICE = 5,           /* a HIP runtime call failed */
    RSVD_ERR_TOO_LARGE = 6,        /* rsvd_solve_noalloc: the problem needs more device scratch
                                      than RSVD_NOALLOC_SCRATCH_BYTES */
    RSVD_ERR_QUEUE_FULL = 7        /* rsvd_server_submit: max_pending requests already wait for
                                      admission; nothing was queued, submit again later */
} rsvd_status;

typedef enum {
    RSVD_F64 = 0,                  /* double: all arithmetic in FP64 (FP64 MFMA) */
    RSVD_F32 = 1,                  /* float: products with A on FP32 MFMA, FP32
                                      accumulation; Gram, Cholesky, small SVD FP64 */
    RSVD_BF16 = 2,                 /* A stored as bfloat16 (uint16 patterns): products on the
                                      BF16 matrix instructions with FP32 accumulation, the other
                                      operand rounded to BF16; everything else as RSVD_F32 */
    RSVD_FP8_E4M3 = 3              /* A stored as FP8 E4M3 (OCP E4M3FN, max 448) with per-column
                                      FP32 scales: A = Aq diag(col_scale); products on the FP8
                                      matrix instructions, FP32 accumulation */
} rsvd_dtype;

/* Bits of the device `info` word written by rsvd_solve / rsvd_orth. */
#define RSVD_INFO_QR_FALLBACK        1  /* CholeskyQR broke down (rank-deficient or
                                           too ill-conditioned Y); Householder QR used */
#define RSVD_INFO_SHIFTED_CHOLESKY   2  /* small SVD: Gram of B singular; a diagonal
                                           shift was used (B rank-deficient) */
#define RSVD_INFO_JACOBI_NOT_CONVERGED 4 /* small SVD hit the sweep cap */
#define RSVD_INFO_NONFINITE          8  /* NaN or Inf met in a Gram matrix */
#define RSVD_INFO_ORTH_BREAKDOWN    16  /* RSVD_ORTH_CHOLQR2: CholeskyQR broke down and no fallback
                                           ran, so a basis is not orthonormal */
#define RSVD_INFO_FALLBACK_TIMEOUT  32  /* a grid barrier of the Householder fallback did not
                                           complete within its wait limit (device oversubscribed);
                                           the basis of that orthonormalisation is not valid */
#define RSVD_INFO_SINGULAR_SYSTEM   64  /* Algorithm 5: the square system of eq. (3.13) has no
                                           usable pivot (Q^T Omega singular or not finite); the
                                           outputs are not valid */

typedef struct rsvd_handle rsvd_handle;

/* Input matrix A: rows x cols, row-major, leading dimension ld (elements),
 * 1 <= rows, cols < 2^31.  A is streamed with 16-byte loads when data is
 * 16-byte aligned and ld is a multiple of 4 (RSVD_F32) or 2 (RSVD_F64);
 * otherwise element loads are used (correct, slower).  RSVD_BF16 and
 * RSVD_FP8_E4M3 data must be 16-byte aligned with ld a multiple of 8 / 16
 * (RSVD_ERR_UNSUPPORTED otherwise); rsvd_quantize produces such matrices.
 *
 * Low-precision forms (the precision layer; the thesis computes in double
 * precision): the power iterations run on the stored A with one extra
 * power iteration by default (rsvd_params.extra_power_pass), and the
 * projection B = Q^T A of Algorithm 4 step 6 (the Rayleigh-Ritz step) uses
 * `master`, an FP32 copy of A, when given; the residual norms need it. */
typedef struct {
    const void* data;
    int32_t dtype;                 /* rsvd_dtype */
    int32_t reserved0;
    int64_t rows, cols, ld;
    const float* col_scale;        /* RSVD_FP8_E4M3: cols scales (device), required; else NULL */
    const float* master;           /* BF16 / FP8: optional FP32 copy of A (device), else NULL */
    int64_t ld_master;             /* leading dimension of master (>= cols) */
} rsvd_matrix;

/* Parameters of Algorithm 4 (inputs A, k, p, q of the algorithm statement). */
typedef struct {
    int64_t k;                     /* target rank, 1 <= k <= min(m, n) */
    int64_t p;                     /* oversampling, p >= 0; l = min(k + p, min(m, n)) */
    int64_t q;                     /* power iterations, q >= 0 (q = 0: Algorithm 2) */
    uint64_t seed;                 /* key of the Philox test matrix */
    int32_t residual;              /* error measure ||A - Q Q^T A|| of Theorems 2, 3, 6 (full l-column Q):
                                      bit 0 (1): spectral norm, estimated (see residual_iters);
                                      bit 1 (2): Frobenius norm, exact (FP64 accumulation); 3: both */
    int32_t return_full_l;         /* 0: return the top k triplets; 1: all l */
    int32_t orth;                  /* orth of Algorithms 1-4: RSVD_ORTH_AUTO (0, CholeskyQR2 with the
                                      Householder fallback on breakdown), RSVD_ORTH_CHOLQR2 (1, CholeskyQR2
                                      only: a breakdown is reported in info, no fallback is enqueued),
                                      RSVD_ORTH_HOUSEHOLDER (2, always Householder QR) */
    int32_t residual_iters;        /* spectral estimate: block power iterations t on E = A - Q Q^T A,
                                      0 = default (4).  Start block: min(16, m, n) columns of the test-matrix
                                      generator on stream 2 (same seed), orthonormalised; each iteration
                                      Y = orth(E Z), Z = orth(E^T Y); the estimate is the largest singular value
                                      of E Z (a lower bound of ||E||_2 up to rounding, converging as t grows).
                                      0 <= residual_iters <= 1000. */
    int32_t extra_power_pass;      /* BF16 / FP8 A: power iterations added to q; -1 = default (1);
                                      ignored for RSVD_F32 / RSVD_F64 */
    int32_t algorithm;             /* 0 or 4: Algorithm 4 (orth after every product of the power scheme);
                                      3: Algorithm 3 (Section 3.2): Y = A Omega, q times Y = A (A^T Y), and
                                      orth only once, after the last product.  In FP32, sigma_1^(2q+1) must
                                      stay inside the float range.
                                      5: Algorithm 5 (Section 3.4.1), single pass, for a symmetric n x n A:
                                      Y = A Omega, Q = orth(Y), C (l x l) from C (Q^T Omega) = Q^T Y
                                      (eq. (3.13), Gauss-Jordan with partial pivoting), the
                                      eigendecomposition of (C + C^T) / 2; S receives the k eigenvalues of
                                      largest magnitude (signed, |S| descending; ties: larger value first),
                                      U their eigenvectors (each column's largest-magnitude entry positive)
                                      and Vt = U^T, so A ~ U diag(S) Vt.  A is read once; its symmetry is
                                      not checked.
                                      6: Algorithm 6 (Section 3.4.2), single pass: Y_c = A Omega_c and
                                      Y_r = A^T Omega_r (Omega_c: the test matrix above, n x l; Omega_r:
                                      the same generator on stream 1, m x l) from one read of A; Q_c, Q_r
                                      the k dominant left singular vectors of Y_c, Y_r; C (k x k) the
                                      least-squares solution of (Omega_r^T Q_c) C = Y_r^T Q_r and
                                      C (Q_r^T Omega_c) = Q_c^T Y_c (eqs. (3.15)-(3.16), equal weights);
                                      U = Q_c U^, V = Q_r V^ from the SVD of C, signs as for Algorithm 4.
                                      Algorithms 5 and 6 need F32 / F64 A, q = 0, l <= 128, the Gaussian
                                      test matrix, return_full_l = 0 and residual = 0
                                      (RSVD_ERR_UNSUPPORTED otherwise); Q, if given, receives orth(Y)
                                      (Algorithm 5) or orth(Y_c) (Algorithm 6), m x l. */
    int32_t jacobi_max_sweeps;     /* sweep cap of the small SVD's Jacobi iteration, 0 = default
                                      (60; 30 for l > 128); reaching it sets RSVD_INFO_JACOBI_NOT_CONVERGED */
    int32_t test_matrix;           /* RSVD_TEST_GAUSSIAN (0): Omega standard Gaussian (rsvd_omega);
                                      RSVD_TEST_SRFT (1): the subsampled randomized trigonometric test
                                      matrix of FastRandRF (Appendix A; see rsvd_srft_omega), generated
                                      in the sketch kernel like the Gaussian one.  F32 / F64 A only. */
    int32_t reserved1;
} rsvd_params;

#define RSVD_TEST_GAUSSIAN 0
#define RSVD_TEST_SRFT 1

#define RSVD_ORTH_AUTO 0
#define RSVD_ORTH_CHOLQR2 1
#define RSVD_ORTH_HOUSEHOLDER 2

/* Outputs.  r = k, or l when return_full_l is set.  U, Vt and Q have the
 * dtype of A (float for BF16 / FP8 A).  S, residual are doubles.  Q
 * (optional) receives the final m x l orthonormal basis of Stage 1. */
typedef struct {
    void* U;  int64_t ldu;         /* m x r, row-major, ldu >= r */
    double* S;                     /* r singular values, descending */
    void* Vt; int64_t ldvt;        /* r x n, row-major, ldvt >= n */
    double* residual;              /* required when params->residual != 0: [0] = spectral estimate,
                                      [1] = Frobenius norm (an entry not requested is 0) */
    int32_t* info;                 /* required; RSVD_INFO_* bit flags */
    void* Q;  int64_t ldq;         /* nullable; m x l, row-major, ldq >= l */
    int32_t* jacobi_sweeps;        /* nullable, device: sweeps run by the small SVD's one-sided Jacobi
                                      iteration (Algorithm 4 step 7), the last of which rotates nothing */
} rsvd_result;

/* Create a handle bound to HIP device `device` (host memory only; the
 * scratch of rsvd_solve and the other calls comes from the caller's
 * workspace, that of rsvd_solve_noalloc from the library's fixed array).
 * *out is NULL on error.
 * Calls made with the handle make `device` current (hipSetDevice); the
 * first rsvd_create on a device also looks up the device address of the
 * scratch array of rsvd_solve_noalloc on it (RSVD_ERR_DEVICE if that fails). */
rsvd_status rsvd_create(rsvd_handle** out, int device);
rsvd_status rsvd_destroy(rsvd_handle* h);

/* l actually used for (m, n, k, p): min(k + p, min(m, n)). */
int64_t rsvd_l_used(int64_t m, int64_t n, int64_t k, int64_t p);

/* Bytes of device workspace rsvd_solve needs for this problem. */
rsvd_status rsvd_workspace_size(const rsvd_handle* h, const rsvd_matrix* A,
                                const rsvd_params* params, size_t* bytes);

/* Enqueue one randomized SVD (Algorithm 4) of A on `stream`.  `workspace`
 * is device memory of at least rsvd_workspace_size bytes, owned by the
 * caller, not used concurrently by another call, 256-byte aligned.  No
 * device memory is allocated by this call. */
rsvd_status rsvd_solve(rsvd_handle* h, const rsvd_matrix* A, const rsvd_params* params,
                       const rsvd_result* out, void* workspace, size_t workspace_bytes,
                       void* stream);

/* Allocation-free form of rsvd_solve, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same arguments, semantics and results
 * as rsvd_solve, except that the workspace is not passed: the solve uses a
 * fixed device scratch array of RSVD_NOALLOC_SCRATCH_BYTES compiled into
 * the library (one copy per device, held from the first rsvd_create on that
 * device until the process ends; its device address is looked up by
 * rsvd_create).  The call itself allocates nothing (no hipMalloc, hipFree
 * or event creation); rsvd_profile_enable does not apply to it.  A problem
 * whose rsvd_workspace_size exceeds RSVD_NOALLOC_SCRATCH_BYTES is refused
 * with RSVD_ERR_TOO_LARGE before anything is enqueued (64 MiB covers, e.g.,
 * 8192 x 8192 FP32 with l = 110).  Every call on one device shares that
 * device's scratch, and a solve initialises the parts it reads: calls that
 * overlap on one device (different streams or host threads without
 * ordering between them) race and give undefined results; calls ordered on
 * one stream are safe. */
#define RSVD_NOALLOC_SCRATCH_BYTES (64ull << 20)
rsvd_status rsvd_solve_noalloc(rsvd_handle* h, const rsvd_matrix* A, const rsvd_params* params,
                               const rsvd_result* out, void* stream);

const char* rsvd_status_string(rsvd_status s);

/* Kernel timing for performance reports.  While enabled, the product kernel
 * of every product with A enqueued by rsvd_solve on handle h is bracketed by
 * a pair of HIP events recorded on the solve's stream (events owned by the
 * handle; the split-K reduction that follows the product is outside them).
 * rsvd_profile_read waits for the recorded events of one kind (0: the
 * sketch A * Omega with the generated test matrix, 1: A * X, 2: A^T * X,
 * 3: all product kinds, 4: the FP32 projection A^T Q on the master copy of a
 * BF16 / FP8 A), returns the summed kernel time in milliseconds and the
 * number of launches, and forgets those records (kind 3 forgets all product
 * records).  Kind 5 is the range finder of each solve (Stage 1 of Algorithm
 * 4: the sketch, the power iterations and every orthonormalisation, from the
 * first kernel after the flag reset to the last orth), one record per solve.
 * Kind 6 is the one-sided Jacobi iteration of the small SVD (Algorithm 4
 * step 7: every kernel of it), one record per solve.  Kind 7 is the
 * two-sided sketch kernel of Algorithm 6 (Y_c = A Omega_c and
 * Y_r = A^T Omega_r from one read of A; the reductions of its partials are
 * outside the events), and it is also counted by kind 3.  For Algorithms 5
 * and 6, kind 5 spans the sketch(es) and their orthonormalisations and
 * kind 6 every small SVD / eigendecomposition of Stage 2. */
rsvd_status rsvd_profile_enable(rsvd_handle* h, int32_t enable);
rsvd_status rsvd_profile_read(rsvd_handle* h, int32_t kind, double* total_ms, int64_t* launches);

/* Low-precision copy of an FP32 matrix (rows x cols, lda) on `stream`:
 * dtype RSVD_BF16: out = uint16 BF16 patterns (round to nearest even), ldo;
 * dtype RSVD_FP8_E4M3: amax_j = max_i |A_ij|, col_scale[j] = amax_j / 448
 * (1 for a zero column), out_ij = e4m3(A_ij * (448 / amax_j)) (round to
 * nearest even, saturating at 448), each division and product rounded in
 * FP32.  All pointers device; col_scale (cols floats) is required for FP8.
 * For use as an rsvd_matrix, out should be 16-byte aligned with ldo a
 * multiple of 8 (BF16) / 16 (FP8). */
rsvd_status rsvd_quantize(int32_t dtype, const float* A, int64_t rows, int64_t cols, int64_t lda, void* out,
                          int64_t ldo, float* col_scale, void* stream);

/* ---- Batched request server: continuous batching on one GPU. ----
 *
 * A server owns a device arena of hbm_budget_bytes (allocated once, at
 * create), n_streams ordinary streams and a scheduler thread.  Submitted
 * requests wait in a queue of at most max_pending entries (0 = 4096; a submit
 * to a full queue returns RSVD_ERR_QUEUE_FULL and queues nothing).  They are
 * admitted oldest first as soon as a stream is free and the request's
 * workspace (rsvd_workspace_size) fits in the arena (admission by HBM
 * footprint).  When the oldest request does not fit, younger requests that
 * fit are admitted past it, but the oldest is passed over at most 8 times;
 * after that admission waits until it fits.  An admitted request is one
 * rsvd_solve on its stream, so requests that arrive while others run overlap
 * on the device.  A request borrows the caller's A and result buffers until
 * it is done; its result is the same as that of rsvd_solve alone.  Submit,
 * poll, wait, release, drain and stats may be called from any thread.  A
 * request whose workspace exceeds the whole arena is refused at submit
 * (RSVD_ERR_NO_MEMORY).  Latency = time from submit until the scheduler sees
 * the request's completion event. */
typedef struct rsvd_server rsvd_server;
rsvd_status rsvd_server_create(rsvd_server** out, int device, size_t hbm_budget_bytes, int n_streams,
                               int32_t max_pending);
/* ready_event (nullable, a hipEvent_t): the request's stream waits for it
 * before the solve's first kernel.  A caller that writes A, or allocates the
 * result buffers, with work on its own stream records an event there after
 * that work and passes it here, so the request never reads A before it is
 * written nor writes a buffer still in use (the server's streams do not
 * synchronise with other streams).  The event is waited on when the request
 * is admitted; it must stay valid until then. */
rsvd_status rsvd_server_submit(rsvd_server* s, const rsvd_matrix* A, const rsvd_params* params,
                               const rsvd_result* out, void* ready_event, uint64_t* ticket);
/* done = 1 once the request's kernels have completed; final_status: its status. */
rsvd_status rsvd_server_poll(rsvd_server* s, uint64_t ticket, int* done, rsvd_status* final_status);
/* Block until the request is done; latency_ms (nullable) receives its latency. */
rsvd_status rsvd_server_wait(rsvd_server* s, uint64_t ticket, rsvd_status* final_status, double* latency_ms);
/* Forget a done request (its ticket becomes unknown): a long-running server
 * holds a record for every request not yet released.  RSVD_ERR_INVALID_ARG
 * for an unknown ticket or a request not done yet. */
rsvd_status rsvd_server_release(rsvd_server* s, uint64_t ticket);
/* paused != 0: admit nothing until called again with 0 (queued requests
 * wait; running ones finish).  For controlled batching and tests. */
rsvd_status rsvd_server_pause(rsvd_server* s, int32_t paused);
/* Block until every submitted request is done. */
rsvd_status rsvd_server_drain(rsvd_server* s);
/* Latency percentiles over the last 65536 completed requests; solves/s =
 * completed / (last completion - first submit); completed counts all. */
rsvd_status rsvd_server_stats(rsvd_server* s, double* p50_ms, double* p99_ms, double* solves_per_s,
                              int64_t* completed);
/* Launch graphs (off by default): each admitted request's kernels are captured
 * into a HIP graph and launched as one.  Executable graphs are pooled by
 * bucket: a request takes an idle graph of its bucket and updates it with its
 * own pointers, sizes and launch grids instead of instantiating a new one;
 * the graph is idle again when the request retires (at most 256 idle graphs
 * are kept, least recently used evicted).  A bucket is what fixes the
 * sequence of kernels: precision, l rounded up to 16, the output width
 * rounded up to 16, q and the options, and whether each product kind is split
 * along its reduction; so requests of different m, n and k share one.  An
 * update the runtime refuses falls back to a new instantiation, and a request
 * whose capture fails is launched directly.  HIP refuses a device-wide
 * synchronisation (hipDeviceSynchronize) from any thread while a stream of the
 * device is capturing: with graphs on, the rest of the process must wait on
 * streams or events instead.  enable = 0 (the default) launches the kernels
 * directly.  Results are the same either way. */
rsvd_status rsvd_server_use_graphs(rsvd_server* s, int32_t enable);
/* Requests launched as graphs so far, executable graphs instantiated
 * (launches minus instantiations = launches that reused an updated graph), and
 * requests launched directly because their capture failed.  Any pointer may be
 * NULL. */
rsvd_status rsvd_server_graph_stats(rsvd_server* s, int64_t* launches, int64_t* instantiations,
                                    int64_t* fallbacks);
/* Drains, then releases the arena, streams, graphs and thread. */
rsvd_status rsvd_server_destroy(rsvd_server* s);

/* ---- Subspace diagnostics and the adaptive range finder ---- */

/* Sines of the canonical angles theta_1 <= ... <= theta_k between range(U1)
 * (rows x k, ld1) and range(U2) (rows x l, ld2), both with orthonormal
 * columns, k <= l <= rows, round16(k) + round16(l) <= 288 (the measure of
 * Section 4.3, eq. (4.3), and of Theorem 5): the singular values of
 * E = (I - U2 U2^T) U1, ascending, written to `sines` (device, k doubles).
 * E is formed from the FP64 Gram of [U2 | U1] (projected twice) and its
 * singular values come from its FP64 Gram, so sines far below
 * sqrt(2^-53) ||E|| (FP64) or the FP32 rounding of U1, U2 (FP32) are not
 * resolved.  dtype F32 or F64; asynchronous on `stream`. */
rsvd_status rsvd_canonical_sines_workspace_size(int32_t dtype, int64_t rows, int64_t k, int64_t l, size_t* bytes);
rsvd_status rsvd_canonical_sines(rsvd_handle* h, int32_t dtype, int64_t rows, int64_t k, const void* U1, int64_t ld1,
                                 int64_t l, const void* U2, int64_t ld2, double* sines, void* workspace,
                                 size_t workspace_bytes, void* stream);

/* Adaptive randomized range finder (Appendix A, Adaptive_randRF), blocked:
 * blocks of `block` (1..32) Gaussian test vectors (columns t*block.. of the
 * test matrix on Philox stream 3, key seed) are drawn until the estimate
 * est = 10 sqrt(2/pi) max_i ||(I - Q Q^T) A w_i|| of the last block is <= tol
 * (then ||(I - Q Q^T) A||_2 <= tol except with probability at most
 * min(m, n) 10^-block).  Each block is projected against Q twice; its left
 * singular vectors with singular value above tol / (10 sqrt(2/pi)) are
 * projected once more, orthonormalised (CholeskyQR2, Householder fallback)
 * and appended.  At most max_l columns (max_l <= min(m, n), round16(max_l) +
 * round16(block) <= 288).  Q (device, m x max_l, ldq >= max_l) receives the
 * l_out columns; est_out the last estimate; converged_out 1 if the
 * tolerance was met, 0 if max_l stopped it.  F32 / F64 A.  Unlike the other
 * calls this one synchronises `stream` once per block (the block count
 * depends on the data) and returns when Q is complete. */
rsvd_status rsvd_adaptive_range_workspace_size(const rsvd_matrix* A, int32_t block, int64_t max_l, size_t* bytes);
rsvd_status rsvd_adaptive_range(rsvd_handle* h, const rsvd_matrix* A, double tol, int32_t block, int64_t max_l,
                                uint64_t seed, void* Q, int64_t ldq, int64_t* l_out, double* est_out,
                                int32_t* converged_out, void* workspace, size_t workspace_bytes, void* stream);

/* ---- Single steps of the path, for testing each kernel on its own. ---- */

/* The test matrix of Algorithm 4 step 1, materialised (the solve never does
 * this).  Element (i, j), 0 <= i < n, 0 <= j < l, comes from the
 * Philox4x32-10 block with counter (i / 4, j, stream_id, 0) and key
 * (seed mod 2^32, seed / 2^32): words (w0, w1) serve rows 4g, 4g+1 and
 * (w2, w3) rows 4g+2, 4g+3; with u1 = ((wa >> 8) + 1) 2^-24 and
 * u2 = (wb >> 8) 2^-24 the even row is sqrt(-2 ln u1) cos(2 pi u2) and the
 * odd row sqrt(-2 ln u1) sin(2 pi u2), evaluated in the precision of
 * `dtype`.  out: n x l row-major, ld >= l. */
rsvd_status rsvd_omega(int32_t dtype, uint64_t seed, uint32_t stream_id, int64_t n, int64_t l,
                       void* out, int64_t ld, void* stream);

/* The SRFT test matrix of FastRandRF (Appendix A: Omega = sqrt(n / l) D F R),
 * materialised (a solve generates it inside the sketch kernel).  Real form:
 * D = diag(d_i), d_i = -1 if bit 0 of word (i mod 4) of the Philox4x32-10
 * block (i / 4, 0, 4, 0) under key (seed) is set, else +1; F the orthonormal
 * DCT-II, F[i][c] = sqrt(2 / n) cos(pi (2 i + 1) c / (2 n)) (sqrt(1 / n) for
 * c = 0); R the l columns c_0 .. c_{l-1} drawn by Floyd's algorithm: step t
 * (j = n - l + t) takes x = floor(w (j + 1) / 2^32), w word 0 of block
 * (t, 1, 4, 0), unless an earlier step took x, else j.  Omega^T Omega =
 * (n / l) I.  out: n x l row-major (ld >= l) of `dtype` (F32 / F64); cols
 * (device, l int32) receives c_0 .. c_{l-1}.  1 <= l <= min(n, 288). */
rsvd_status rsvd_srft_omega(int32_t dtype, uint64_t seed, int64_t n, int64_t l, void* out, int64_t ld,
                            int32_t* cols, void* stream);

/* Raw Philox4x32-10 words: for each of `count` counter pairs (g, j) in
 * ctr (device, 2*count uint32), writes the 4 words of block
 * (g, j, stream_id, 0) under key (seed) to out (device, 4*count uint32). */
rsvd_status rsvd_philox_words(uint64_t seed, uint32_t stream_id, const uint32_t* ctr, int64_t count,
                              uint32_t* out, void* stream);

/* Y = A X (trans = 0; X is n x ncols, Y is m x ncols) or Y = A^T X
 * (trans = 1; X is m x ncols, Y is n x ncols) with the solve's MFMA kernels.
 * If X is NULL and trans = 0, X is the test matrix Omega(seed) (generated in
 * the kernel).  ncols <= 288.  For BF16 / FP8 A, X and Y are float and X is
 * rounded to A's format first (FP8: rows of X scaled by col_scale for
 * trans = 0, then per-column scales t_c = amax_c / 448), exactly as in a
 * solve.  Uses `workspace` (rsvd_gemm_workspace_size). */
rsvd_status rsvd_gemm_workspace_size(const rsvd_matrix* A, int32_t trans, int64_t ncols, size_t* bytes);
rsvd_status rsvd_gemm(rsvd_handle* h, const rsvd_matrix* A, int32_t trans, const void* X, int64_t ldx,
                      uint64_t seed, int64_t ncols, void* Y, int64_t ldy,
                      void* workspace, size_t workspace_bytes, void* stream);

/* Two-sided sketch of the single-pass Algorithm 6 (step 2): Y_c = A Omega_c
 * (m x l, ldyc >= l) and Y_r = A^T Omega_r (n x l, ldyr >= l) from one read
 * of A (F32 / F64), with the kernel of the solve.  Omega_c is the test
 * matrix of rsvd_omega(seed, stream 0) (n x l), Omega_r that of stream 1
 * (m x l).  omega_c (n x l, ldoc >= l) and omega_r (m x l, ldor >= l), when
 * not NULL, receive the two test matrices as the kernel generated them.
 * 1 <= l <= 128.  Uses `workspace` (rsvd_dual_sketch_workspace_size). */
rsvd_status rsvd_dual_sketch_workspace_size(const rsvd_matrix* A, int64_t l, size_t* bytes);
rsvd_status rsvd_dual_sketch(rsvd_handle* h, const rsvd_matrix* A, uint64_t seed, int64_t l, void* Yc,
                             int64_t ldyc, void* Yr, int64_t ldyr, void* omega_c, int64_t ldoc, void* omega_r,
                             int64_t ldor, void* workspace, size_t workspace_bytes, void* stream);

/* orth of Algorithms 1-4: Q (rows x l, ldq) = orthonormal basis of range(Y)
 * (rows x l, ldy), l <= rows, by CholeskyQR2 (FP64 Gram and Cholesky) with a
 * Householder QR fallback; diag(R) > 0 so Q is the Q factor of the thin QR.
 * orth_mode: RSVD_ORTH_AUTO, RSVD_ORTH_CHOLQR2 or RSVD_ORTH_HOUSEHOLDER (as
 * rsvd_params.orth).  For FP32 Y the second CholeskyQR pass is skipped when
 * the first factor shows that the first pass is already orthonormal to
 * within 2^-24.  info: device int32, receives the RSVD_INFO_* flags. */
rsvd_status rsvd_orth_workspace_size(int32_t dtype, int64_t rows, int64_t l, size_t* bytes);
rsvd_status rsvd_orth(rsvd_handle* h, int32_t dtype, int64_t rows, int64_t l, const void* Y, int64_t ldy,
                      void* Q, int64_t ldq, int32_t orth_mode, int32_t* info,
                      void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RSVD_H */
