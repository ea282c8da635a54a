// Host driver of the C ABI (include/rsvd.h): argument checks, workspace
// layout and the launch sequence of Algorithm 4 on one HIP stream.
//
// A solve is a fixed chain of kernels on the caller's stream; nothing in it
// synchronises with the host.  Data-dependent choices (the Householder
// fallback of orth, the shifted Cholesky of the small SVD) are taken on the
// device through flags in the workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rsvd.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace rsvd;

struct rsvd_handle {
    int device;
    // Optional timing of the products with A (rsvd_profile_*): one event pair
    // per launch, recorded on the solve's stream around the kernel.
    bool profiling = false;
    struct Rec { int kind; hipEvent_t start, stop; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get_event() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

// Device scratch of the allocation-free entry point rsvd_solve_noalloc: a
// file-scope array of kScratchBytes in every device's copy of this code
// object.  Its name is only a host-side stand-in; host code uses the device
// address that hipGetSymbolAddress returns for the device (scratch_ptr).
constexpr size_t kScratchBytes = (size_t)RSVD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Look up (once per device, with that device current) the device address of
// the scratch array.
hipError_t scratch_init(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255)) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void* scratch_ptr(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

constexpr size_t kAlign = 256;

size_t esize(int dtype) { return dtype == RSVD_F64 ? 8 : 4; }
bool is_lowp(int dtype) { return dtype == RSVD_BF16 || dtype == RSVD_FP8_E4M3; }
int lowp_bytes(int dtype) { return dtype == RSVD_BF16 ? 2 : 1; }
// Working precision of the panels (Y, Q, W, U, V): float for BF16 / FP8 A.
int work_dtype(int dtype) { return is_lowp(dtype) ? RSVD_F32 : dtype; }

struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += (bytes + kAlign - 1) / kAlign * kAlign;
        return o;
    }
};

// Workspace of one solve (offsets in bytes from the workspace base).
struct Plan {
    int dtype = 1;
    int64_t m = 0, n = 0, k = 0, p = 0, q = 0, l = 0, r = 0;
    int L = 0;
    int ncounters = 0;
    int splits_nn = 1, splits_tn = 1;
    size_t counters, flags, part, Y, Q, W, GP, R, Rinv, Ut, Mv, sigma, shift, sign, amax_val, amax_idx, H, Qw,
        work, res_part, res, cols;
    // Low-precision A: format, prepared operand (L x ldt) and its scales.
    int afmt = 0;
    int splits_lp_nn = 1, splits_lp_tn = 1;
    int64_t ldt = 0;
    size_t Xt = 0, tsc = 0, amax = 0, smax = 0;
    // Spectral-norm estimator of the residual (allocated when requested):
    // block of sb <= 16 columns padded to 16.
    int spectral = 0, sb = 0;
    int splits16_nn = 1, splits16_tn = 1;
    size_t flags2 = 0, QW = 0, Za = 0, Zb = 0, Ws = 0, Ys = 0, Mc = 0, sigma2 = 0, shift2 = 0;
    size_t total;
};

constexpr int kSpecBlock = 16;      // block size of the spectral-norm estimator
constexpr int kSpecItersDefault = 4;

bool make_plan(int adtype, int64_t m, int64_t n, int64_t k, int64_t p, int64_t q, int full, Plan& P,
               int spectral = 0) {
    const int dtype = work_dtype(adtype);
    P.afmt = adtype;
    P.dtype = dtype;
    P.m = m; P.n = n; P.k = k; P.p = p; P.q = q;
    P.l = std::min<int64_t>(k + p, std::min(m, n));
    P.r = full ? P.l : k;
    P.L = (int)round_up(P.l, 16);
    if (P.L > kMaxL) return false;
    const int64_t mx = std::max(m, n);
    const size_t es = esize(dtype);
    const size_t pn = gemm_partials_elems(dtype, m, n, P.L, &P.splits_nn);
    const size_t pt = gemm_partials_elems(dtype, n, m, P.L, &P.splits_tn);
    P.spectral = spectral;
    P.sb = (int)std::min<int64_t>(kSpecBlock, std::min(m, n));
    const size_t pn16 = spectral ? gemm_partials_elems(dtype, m, n, kSpecBlock, &P.splits16_nn) : 0;
    const size_t pt16 = spectral ? gemm_partials_elems(dtype, n, m, kSpecBlock, &P.splits16_tn) : 0;
    P.ncounters = 1;
    Carver c;
    P.counters = c.take(sizeof(int) * (size_t)P.ncounters);
    P.flags = c.take(sizeof(DevFlags));
    size_t plp = 0;
    if (is_lowp(adtype)) {
        plp = std::max(lp_partials_elems(m, n, P.L, &P.splits_lp_nn), lp_partials_elems(n, m, P.L, &P.splits_lp_tn));
        P.ldt = round_up(mx, 64);
    }
    // The split-K partials are idle during an orthonormalisation, so the
    // Householder fallback's tree levels share their space.
    P.part = c.take(std::max(es * std::max<size_t>({pn, pt, pn16, pt16, plp, 1}),
                             sizeof(double) * householder_scratch_doubles(mx, P.L)));
    P.Y = c.take(es * (size_t)mx * P.L);
    P.Q = c.take(es * (size_t)m * P.L);
    P.W = c.take(es * (size_t)n * P.L);
    P.GP = c.take(sizeof(double) * std::max(gram_partials_elems(mx, P.L),
                                            spectral ? gram_partials_elems(m, P.L + kSpecBlock) : 0));
    P.R = c.take(sizeof(double) * (size_t)P.L * P.L);
    P.Rinv = c.take(sizeof(double) * (size_t)P.L * P.L);
    P.Ut = c.take(sizeof(double) * (size_t)P.L * P.L);
    P.Mv = c.take(sizeof(double) * (size_t)P.L * P.L);
    P.sigma = c.take(sizeof(double) * (size_t)P.L);
    P.shift = c.take(sizeof(double));
    P.sign = c.take(sizeof(double) * (size_t)P.L);
    P.amax_val = c.take(sizeof(double) * (size_t)apply_blocks(n) * P.L);
    P.amax_idx = c.take(sizeof(int) * (size_t)apply_blocks(n) * P.L);
    P.H = c.take(sizeof(double) * (size_t)mx * P.L);
    P.Qw = c.take(sizeof(double) * (size_t)mx * P.L);
    P.work = c.take(sizeof(double) * kJacobiWorkDoubles);
    P.res_part = c.take(sizeof(double) * residual_partials(m, n));
    P.res = c.take(sizeof(double) * 2);
    P.cols = c.take(sizeof(int) * (size_t)P.L);
    if (is_lowp(adtype)) {
        P.Xt = c.take((size_t)lowp_bytes(adtype) * (size_t)P.L * (size_t)P.ldt);
        P.tsc = c.take(sizeof(float) * (size_t)P.L);
        P.amax = c.take(sizeof(unsigned) * (size_t)P.L);
        P.smax = c.take(sizeof(float));
    }
    if (spectral) {
        P.flags2 = c.take(sizeof(DevFlags));
        P.QW = c.take(es * (size_t)m * (P.L + kSpecBlock));
        P.Za = c.take(es * (size_t)n * kSpecBlock);
        P.Zb = c.take(es * (size_t)n * kSpecBlock);
        P.Ws = c.take(es * (size_t)m * kSpecBlock);
        P.Ys = c.take(es * (size_t)m * kSpecBlock);
        P.Mc = c.take(sizeof(double) * (size_t)(P.L + kSpecBlock) * kSpecBlock);
        P.sigma2 = c.take(sizeof(double) * kSpecBlock);
        P.shift2 = c.take(sizeof(double));
    }
    P.total = c.off;
    return true;
}

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

#define RSVD_TRY(expr)                                     \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return RSVD_ERR_DEVICE;      \
    } while (0)

// The second CholeskyQR pass is switched off when the first one is already
// orthonormal to within 2^-24 (FP32 panels; see chol_finish_orth): a second
// pass could then only move Q by less than its storage precision.  FP64
// panels always take it.
constexpr double kPass2SkipTauF32 = 0x1.0p-24;

// Rotation threshold of the small SVD's one-sided Jacobi iteration (a pair
// rotates while |x_i . x_j| > tol |x_i| |x_j|).  FP64 data: 1e-15, columns
// orthogonal to the working precision.  FP32 and lower-precision data, whose
// own rounding is at least 2^-24 relative: 2^-34, so the columns' remaining
// non-orthogonality (which perturbs the singular values only to second order)
// stays three decades below the data's precision; this saves the last sweep
// of the quadratically convergent iteration.
constexpr double kJacobiTolF64 = 1e-15;
constexpr double kJacobiTolLow = 0x1.0p-34;
double jacobi_tol(int dtype) { return dtype == RSVD_F64 ? kJacobiTolF64 : kJacobiTolLow; }

// orth(Y) -> Q for an internal rows x L buffer (ld = L, l valid columns,
// zero padding), with the outcome in `flags`.  Qout must not alias Y.
// CholeskyQR2: Q1 = Y R1^{-1} is written to Qout, and the second pass
// multiplies Qout by R2^{-1} in place.
rsvd_status run_orth_cols(const Plan& P, void* ws, DevFlags* flags, int dtype, int64_t rows, int l, int L,
                          const void* Y, void* Qout, int orth_mode, hipStream_t s, int64_t ldy = 0) {
    if (ldy == 0) ldy = L;
    double* R = at<double>(ws, P.R);
    double* Rinv = at<double>(ws, P.Rinv);
    double* GP = at<double>(ws, P.GP);
    double* work = at<double>(ws, P.work);
    if (orth_mode != RSVD_ORTH_HOUSEHOLDER) {
        const int report = orth_mode == RSVD_ORTH_CHOLQR2;
        const double skip_tau = dtype == RSVD_F32 ? kPass2SkipTauF32 : 0.0;
        RSVD_TRY(launch_gram(dtype, Y, ldy, rows, L, GP, nullptr, s));
        RSVD_TRY(launch_chol(GP, rows, l, L, R, Rinv, flags, 0, nullptr, work, 0.0, s, skip_tau, report));
        RSVD_TRY(launch_apply(dtype, Y, ldy, rows, L, Rinv, L, L, Qout, L, 0, nullptr, &flags->orth_fail, nullptr,
                              nullptr, 1, s));
        RSVD_TRY(launch_gram(dtype, Qout, L, rows, L, GP, &flags->pass2_off, s));
        RSVD_TRY(launch_chol(GP, rows, l, L, R, Rinv, flags, 1, nullptr, work,
                             dtype == RSVD_F64 ? 0x1.0p-26 : 0x1.0p-13, s, 0.0, report));
        RSVD_TRY(launch_apply(dtype, Qout, L, rows, L, Rinv, L, L, Qout, L, 0, nullptr, &flags->pass2_off, nullptr,
                              nullptr, 1, s));
        if (orth_mode == RSVD_ORTH_CHOLQR2) return RSVD_OK;
    }
    RSVD_TRY(launch_householder(dtype, Y, ldy, rows, l, L, Qout, L, at<double>(ws, P.H), at<double>(ws, P.Qw),
                                at<double>(ws, P.part), flags, orth_mode == RSVD_ORTH_HOUSEHOLDER, s));
    return RSVD_OK;
}

rsvd_status run_orth(const Plan& P, void* ws, int dtype, int64_t rows, const void* Y, void* Qout, int orth_mode,
                     hipStream_t s) {
    return run_orth_cols(P, ws, at<DevFlags>(ws, P.flags), dtype, rows, (int)P.l, P.L, Y, Qout, orth_mode, s);
}

// Product of A with a skinny block: Yout (ldy) = A X or A^T X, X with ldx
// and `cols` columns (zero padded to `wcols`), or X = Omega(seed) when NULL.
// Timed (rsvd_profile_*) when h is not NULL and profiling is on.
rsvd_status run_product(rsvd_handle* h, const Plan& P, void* ws, const rsvd_matrix* A, int trans, const void* X,
                        int64_t ldx, uint64_t seed, int cols, int wcols, int splits, void* Yout, int64_t ldy,
                        hipStream_t s, int kind = -1, const int* srft_cols = nullptr) {
    GemmArgs g{};
    g.omega_kind = srft_cols ? kOmegaSrft : kOmegaGaussian;
    g.srft_cols = srft_cols;
    g.A = A->data;
    g.lda = A->ld;
    g.trans = trans;
    g.M = trans ? A->cols : A->rows;
    g.K = trans ? A->rows : A->cols;
    g.X = X;
    g.ldx = ldx;
    g.seed = seed;
    g.ncols = cols;
    g.wcols = wcols;
    g.Y = Yout;
    g.ldy = ldy;
    g.partials = at<char>(ws, P.part);
    g.splits = splits;
    if (!h || !h->profiling) {
        RSVD_TRY(launch_gemm(P.dtype, g, s));
        return RSVD_OK;
    }
    rsvd_handle::Rec rec{kind >= 0 ? kind : (trans ? 2 : (X ? 1 : 0)), nullptr, nullptr};
    rec.start = h->get_event();
    rec.stop = h->get_event();
    if (!rec.start || !rec.stop) return RSVD_ERR_DEVICE;
    RSVD_TRY(hipEventRecord(rec.start, s));
    RSVD_TRY(launch_gemm(P.dtype, g, s, rec.stop));
    h->recs.push_back(rec);
    return RSVD_OK;
}

// Product with a BF16 / FP8 A on the solve's L-column float buffers: the
// operand is rounded to A's format (and transposed) first, the test matrix
// is generated in the kernel.
rsvd_status run_product_lowp(rsvd_handle* h, const Plan& P, void* ws, const rsvd_matrix* A, int trans,
                             const void* X, uint64_t seed, void* Yout, hipStream_t s) {
    const int fmt = A->dtype;
    LpGemmArgs a{};
    a.A = A->data;
    a.lda = A->ld;
    a.col_scale = fmt == RSVD_FP8_E4M3 ? A->col_scale : nullptr;
    a.trans = trans;
    a.M = trans ? A->cols : A->rows;
    a.K = trans ? A->rows : A->cols;
    a.seed = seed;
    a.ncols = X ? P.L : (int)P.l;
    a.wcols = P.L;
    a.Y = static_cast<float*>(Yout);
    a.ldy = P.L;
    a.partials = at<float>(ws, P.part);
    a.splits = trans ? P.splits_lp_tn : P.splits_lp_nn;
    a.ldt = P.ldt;
    if (X) {
        float* tsc = at<float>(ws, P.tsc);
        RSVD_TRY(launch_lp_operand(fmt, static_cast<const float*>(X), a.K, P.L, P.L,
                                   (fmt == RSVD_FP8_E4M3 && !trans) ? A->col_scale : nullptr, at<char>(ws, P.Xt),
                                   P.ldt, P.L, tsc, at<unsigned>(ws, P.amax), s));
        a.Xt = at<char>(ws, P.Xt);
        a.xscale = fmt == RSVD_FP8_E4M3 ? tsc : nullptr;
    } else {
        a.omega_scale = fmt == RSVD_FP8_E4M3 ? at<float>(ws, P.smax) : nullptr;
    }
    if (!h || !h->profiling) {
        RSVD_TRY(launch_lp_gemm(fmt, a, s));
        return RSVD_OK;
    }
    rsvd_handle::Rec rec{trans ? 2 : (X ? 1 : 0), h->get_event(), h->get_event()};
    if (!rec.start || !rec.stop) return RSVD_ERR_DEVICE;
    RSVD_TRY(hipEventRecord(rec.start, s));
    RSVD_TRY(launch_lp_gemm(fmt, a, s, rec.stop));
    h->recs.push_back(rec);
    return RSVD_OK;
}

// The products of Algorithm 4 on the solve's L-column buffers.
// srft_cols: the sketch uses the SRFT test matrix with these sampled columns.
rsvd_status run_gemm(rsvd_handle* h, const Plan& P, void* ws, const rsvd_matrix* A, int trans, const void* X,
                     uint64_t seed, void* Yout, hipStream_t s, int kind = -1, const int* srft_cols = nullptr) {
    if (is_lowp(A->dtype)) return run_product_lowp(h, P, ws, A, trans, X, seed, Yout, s);
    const int cols = trans ? P.L : (X ? P.L : (int)P.l);
    return run_product(h, P, ws, A, trans, X, P.L, seed, cols, P.L, trans ? P.splits_tn : P.splits_nn, Yout, P.L, s,
                       kind, X ? nullptr : srft_cols);
}

// The FP32 copy of a low-precision A (for the Rayleigh-Ritz projection and
// the residual), as a matrix of its own.
rsvd_matrix master_view(const rsvd_matrix* A) {
    rsvd_matrix M{};
    M.data = A->master;
    M.dtype = RSVD_F32;
    M.rows = A->rows;
    M.cols = A->cols;
    M.ld = A->ld_master;
    return M;
}

// ||A - Q Q^T A||_2 estimated by block power iteration on E = A - Q Q^T A
// (the error measure of Theorems 2, 3 and 6): Z_0 = orth(Omega) with the
// test-matrix generator on stream 2 (sb columns); `iters` times
// Y = orth(E Z), Z = orth(E^T Y); then the largest singular value of E Z
// (Rayleigh-Ritz on the final block).  E Z = A Z - Q (Q^T A Z) in FP64 from
// the Gram of [Q | A Z]; E^T Y = A^T Y because Y is orthogonal to Q.  All
// orthonormalisations report into a flag word of their own, so a fallback
// here never shows in the solve's info.
rsvd_status run_spectral(const Plan& P, void* ws, const rsvd_matrix* A, const void* Q, uint64_t seed, int iters,
                         double* out, int fro_requested, hipStream_t s) {
    const int dt = P.dtype, L = P.L, LW = P.L + kSpecBlock, b = P.sb, B = kSpecBlock;
    const size_t es = esize(dt);
    DevFlags* f2 = at<DevFlags>(ws, P.flags2);
    char* QW = at<char>(ws, P.QW);
    void* Za = at<char>(ws, P.Za);
    void* Zb = at<char>(ws, P.Zb);
    void* Wsp = at<char>(ws, P.Ws);
    void* Ys = at<char>(ws, P.Ys);
    double* Mc = at<double>(ws, P.Mc);
    double* GP = at<double>(ws, P.GP);
    RSVD_TRY(launch_init(nullptr, 0, f2, s));
    RSVD_TRY(launch_copy2d(dt, Q, L, P.m, L, QW, LW, L, s));                 // [Q | .]
    if (b < B) RSVD_TRY(launch_copy2d(dt, Za, B, P.n, 0, Za, B, B, s));    // zero padding columns
    RSVD_TRY(launch_omega(dt, seed, 2, P.n, b, Za, B, s));
    rsvd_status st;
    if ((st = run_orth_cols(P, ws, f2, dt, P.n, b, B, Za, Zb, 0, s)) != RSVD_OK) return st;
    // E Z for the block in Zb -> Wsp.
    auto apply_E = [&]() -> rsvd_status {
        rsvd_status r = run_product(nullptr, P, ws, A, 0, Zb, B, 0, B, B, P.splits16_nn, QW + es * L, LW, s);
        if (r != RSVD_OK) return r;
        RSVD_TRY(launch_gram(dt, QW, LW, P.m, LW, GP, nullptr, s));
        RSVD_TRY(launch_proj_coef(GP, P.m, L, b, Mc, s));
        RSVD_TRY(launch_apply(dt, QW, LW, P.m, LW, Mc, B, B, Wsp, B, 0, nullptr, nullptr, nullptr, nullptr, 0, s));
        return RSVD_OK;
    };
    for (int it = 0; it < iters; ++it) {
        if ((st = apply_E()) != RSVD_OK) return st;
        if ((st = run_orth_cols(P, ws, f2, dt, P.m, b, B, Wsp, Ys, 0, s)) != RSVD_OK) return st;
        if ((st = run_product(nullptr, P, ws, A, 1, Ys, B, 0, B, B, P.splits16_tn, Za, B, s)) != RSVD_OK) return st;
        if ((st = run_orth_cols(P, ws, f2, dt, P.n, b, B, Za, Zb, 0, s)) != RSVD_OK) return st;
    }
    if ((st = apply_E()) != RSVD_OK) return st;
    // Rayleigh-Ritz: singular values of E Z (m x b) through its Gram, as for B.
    double* sigma2 = at<double>(ws, P.sigma2);
    double* shift2 = at<double>(ws, P.shift2);
    RSVD_TRY(launch_gram(dt, Wsp, B, P.m, B, GP, nullptr, s));
    RSVD_TRY(launch_chol(GP, P.m, b, B, at<double>(ws, P.R), at<double>(ws, P.Rinv), f2, 2, shift2,
                         at<double>(ws, P.work), 0.0, s));
    RSVD_TRY(launch_jacobi(at<double>(ws, P.R), b, B, shift2, sigma2, at<double>(ws, P.Ut), at<double>(ws, P.Mv), f2,
                           at<double>(ws, P.work), jacobi_tol(dt), s));
    RSVD_TRY(launch_residual_spec_final(sigma2, out, fro_requested, s));
    return RSVD_OK;
}

rsvd_status check_matrix(const rsvd_matrix* A) {
    if (!A || !A->data) return RSVD_ERR_INVALID_ARG;
    if (A->dtype != RSVD_F32 && A->dtype != RSVD_F64 && !is_lowp(A->dtype)) return RSVD_ERR_INVALID_ARG;
    if (A->rows < 1 || A->cols < 1 || A->ld < A->cols) return RSVD_ERR_INVALID_ARG;
    if (A->rows > (int64_t)1 << 31 || A->cols > (int64_t)1 << 31) return RSVD_ERR_UNSUPPORTED;
    if (is_lowp(A->dtype)) {
        if (A->dtype == RSVD_FP8_E4M3 && !A->col_scale) return RSVD_ERR_INVALID_ARG;
        if (A->master && A->ld_master < A->cols) return RSVD_ERR_INVALID_ARG;
        if ((reinterpret_cast<uintptr_t>(A->data) & 15) || (A->ld * lowp_bytes(A->dtype)) % 16)
            return RSVD_ERR_UNSUPPORTED;
    }
    return RSVD_OK;
}

rsvd_status check_params(const rsvd_matrix* A, const rsvd_params* p) {
    if (!p) return RSVD_ERR_INVALID_ARG;
    const int64_t mn = std::min(A->rows, A->cols);
    if (p->k < 1 || p->k > mn || p->p < 0 || p->q < 0 || p->q > 64) return RSVD_ERR_INVALID_ARG;
    if (p->residual < 0 || p->residual > 3 || p->residual_iters < 0 || p->residual_iters > 1000)
        return RSVD_ERR_INVALID_ARG;
    if (p->extra_power_pass < -1 || p->extra_power_pass > 8) return RSVD_ERR_INVALID_ARG;
    if (p->orth < RSVD_ORTH_AUTO || p->orth > RSVD_ORTH_HOUSEHOLDER) return RSVD_ERR_INVALID_ARG;
    if (p->algorithm != 0 && (p->algorithm < 3 || p->algorithm > 6)) return RSVD_ERR_INVALID_ARG;
    if (p->jacobi_max_sweeps < 0 || p->jacobi_max_sweeps > 1000) return RSVD_ERR_INVALID_ARG;
    if (p->test_matrix != RSVD_TEST_GAUSSIAN && p->test_matrix != RSVD_TEST_SRFT) return RSVD_ERR_INVALID_ARG;
    if (p->test_matrix == RSVD_TEST_SRFT && is_lowp(A->dtype)) return RSVD_ERR_UNSUPPORTED;
    if (is_lowp(A->dtype) && p->residual && !A->master) return RSVD_ERR_INVALID_ARG;
    if (round_up(std::min<int64_t>(p->k + p->p, mn), 16) > kMaxL) return RSVD_ERR_UNSUPPORTED;
    return RSVD_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Single-pass Algorithms 5 and 6: the limits of their kernels.
constexpr int kMaxSingleL = 128;
constexpr uint32_t kOmegaRowStream = 1;      // Omega_r of Algorithm 6
bool single_pass(const rsvd_params* p) { return p->algorithm == 5 || p->algorithm == 6; }

rsvd_status check_single_pass(const rsvd_matrix* A, const rsvd_params* p) {
    if (A->dtype != RSVD_F32 && A->dtype != RSVD_F64) return RSVD_ERR_UNSUPPORTED;
    if (p->q != 0 || p->test_matrix != RSVD_TEST_GAUSSIAN || p->return_full_l || p->residual)
        return RSVD_ERR_UNSUPPORTED;
    if (p->algorithm == 5 && A->rows != A->cols) return RSVD_ERR_INVALID_ARG;
    if (std::min<int64_t>(p->k + p->p, std::min(A->rows, A->cols)) > kMaxSingleL) return RSVD_ERR_UNSUPPORTED;
    return RSVD_OK;
}

// Workspace bytes of a single-pass solve (defined with its layout below).
rsvd_status sp_workspace_bytes(const rsvd_matrix* A, const rsvd_params* p, size_t* bytes);


}  // namespace

extern "C" {

const char* rsvd_status_string(rsvd_status s) {
    switch (s) {
        case RSVD_OK: return "ok";
        case RSVD_ERR_INVALID_ARG: return "invalid argument";
        case RSVD_ERR_UNSUPPORTED: return "unsupported request";
        case RSVD_ERR_NO_MEMORY: return "out of memory";
        case RSVD_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case RSVD_ERR_DEVICE: return "HIP runtime error";
        case RSVD_ERR_TOO_LARGE:
            return "problem needs more device scratch than rsvd_solve_noalloc holds (RSVD_NOALLOC_SCRATCH_BYTES)";
        case RSVD_ERR_QUEUE_FULL: return "server queue full (max_pending requests wait for admission)";
    }
    return "unknown status";
}

int64_t rsvd_l_used(int64_t m, int64_t n, int64_t k, int64_t p) { return std::min(k + p, std::min(m, n)); }

rsvd_status rsvd_create(rsvd_handle** out, int device) {
    if (!out) return RSVD_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return RSVD_ERR_DEVICE;
    if (device < 0 || device >= count) return RSVD_ERR_INVALID_ARG;
    if (device >= kMaxDevices) return RSVD_ERR_UNSUPPORTED;
    if (scratch_init(device) != hipSuccess) return RSVD_ERR_DEVICE;
    rsvd_handle* h = new (std::nothrow) rsvd_handle;
    if (!h) return RSVD_ERR_NO_MEMORY;
    h->device = device;
    *out = h;
    return RSVD_OK;
}

rsvd_status rsvd_destroy(rsvd_handle* h) {
    if (!h) return RSVD_OK;
    for (auto& r : h->recs) { h->pool.push_back(r.start); h->pool.push_back(r.stop); }
    for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
    delete h;
    return RSVD_OK;
}

rsvd_status rsvd_profile_enable(rsvd_handle* h, int32_t enable) {
    if (!h) return RSVD_ERR_INVALID_ARG;
    h->profiling = enable != 0;
    return RSVD_OK;
}

rsvd_status rsvd_profile_read(rsvd_handle* h, int32_t kind, double* total_ms, int64_t* launches) {
    if (!h || !total_ms || !launches || kind < 0 || kind > 7) return RSVD_ERR_INVALID_ARG;
    double tot = 0.0;
    int64_t cnt = 0;
    std::vector<rsvd_handle::Rec> keep;
    for (auto& r : h->recs) {
        const bool match = kind == 3 ? (r.kind <= 2 || r.kind == 4 || r.kind == 7) : r.kind == kind;   // kind 3: every product
        if (!match) { keep.push_back(r); continue; }
        if (hipEventSynchronize(r.stop) != hipSuccess) return RSVD_ERR_DEVICE;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return RSVD_ERR_DEVICE;
        tot += ms;
        ++cnt;
        h->pool.push_back(r.start);
        h->pool.push_back(r.stop);
    }
    h->recs.swap(keep);
    *total_ms = tot;
    *launches = cnt;
    return RSVD_OK;
}

rsvd_status rsvd_workspace_size(const rsvd_handle* h, const rsvd_matrix* A, const rsvd_params* params,
                                size_t* bytes) {
    (void)h;
    if (!bytes) return RSVD_ERR_INVALID_ARG;
    rsvd_status st = check_matrix(A);
    if (st != RSVD_OK) return st;
    if ((st = check_params(A, params)) != RSVD_OK) return st;
    if (single_pass(params)) return sp_workspace_bytes(A, params, bytes);
    Plan P;
    if (!make_plan(A->dtype, A->rows, A->cols, params->k, params->p, params->q, params->return_full_l, P,
                   params->residual & 1))
        return RSVD_ERR_UNSUPPORTED;
    *bytes = P.total;
    return RSVD_OK;
}

}  // extern "C"

namespace {

// ------------------------------------------------------------------------
// Single-pass Algorithms 5 and 6 (Section 3.4).

// Workspace: the Plan of Algorithm 4 for the same shape (flags, orth
// scratch, Q = Q_1 (m x L), W = Q_2 (n x L), small-SVD buffers), then the
// panels [Omega_r | Y_c] (m x 2L) and [Y_r | Omega_c] or [Y | Omega]
// (n x 2L), the sketch partials and the FP64 Stage 2 matrices.
struct SpLayout {
    Plan base;
    int alg = 6, Lk = 16, splits = 1, tiles = 1;
    // Pairs solved by one two-problem small-SVD launch sit side by side:
    // Ut_c, Ut_r (L x L each), UtP, UtS (Lk x Lk each) and their sigmas,
    // factors, shifts and Mv scratch.
    size_t part_c = 0, part_r = 0, panel_m = 0, panel_n = 0, xpart = 0, CTc = 0, CTr = 0, X = 0, Ut_cr = 0,
           UtPS = 0, UtC = 0, MvC = 0, sig_cr = 0, sigPS = 0, sigC = 0, R2 = 0, shift2 = 0, Mv2 = 0,
           lam = 0, G1 = 0, G2 = 0, F = 0, T1 = 0, Cm = 0, T2 = 0, Ct = 0, T3 = 0, Wu = 0, Wv = 0, shiftE = 0,
           total = 0;
};

bool sp_layout(int dtype, int alg, int64_t m, int64_t n, int64_t k, int64_t p, SpLayout& S) {
    Plan& P = S.base;
    if (!make_plan(dtype, m, n, k, p, 0, 0, P)) return false;
    if (P.l > kMaxSingleL) return false;
    S.alg = alg;
    const int L = P.L;
    const int Lk = S.Lk = (int)round_up(k, 16);
    const size_t es = esize(dtype), d8 = sizeof(double);
    Carver c;
    c.take(P.total);                                        // the base plan sits at offset 0
    if (alg == 6) {
        S.splits = dual_splits(dtype, m, n);
        S.tiles = dual_row_tiles(dtype, m);
        S.part_c = c.take(es * (S.splits > 1 ? (size_t)S.splits * m * L : 1));
        S.part_r = c.take(es * (size_t)S.tiles * n * L);
        S.panel_m = c.take(es * (size_t)m * 2 * L);
    }
    S.panel_n = c.take(es * (size_t)n * 2 * L);
    S.xpart = c.take(d8 * cross_partials_elems(std::max(m, n), 2 * L, L));
    S.CTc = c.take(d8 * 2 * L * L);
    S.sigC = c.take(d8 * L);
    S.lam = c.take(d8 * L);
    S.Wu = c.take(d8 * (size_t)L * Lk);
    S.shiftE = c.take(d8);
    if (alg == 5) {
        S.X = c.take(d8 * (size_t)L * L);
    } else {
        S.CTr = c.take(d8 * 2 * L * L);
        S.Ut_cr = c.take(d8 * 2 * (size_t)L * L);
        S.UtPS = c.take(d8 * 2 * (size_t)Lk * Lk);
        for (size_t* f : {&S.UtC, &S.MvC, &S.F, &S.T1, &S.Cm, &S.T2, &S.Ct, &S.T3})
            *f = c.take(d8 * (size_t)Lk * Lk);
        S.sig_cr = c.take(d8 * 2 * L);
        S.sigPS = c.take(d8 * 2 * Lk);
        S.R2 = c.take(d8 * 2 * (size_t)L * L);
        S.Mv2 = c.take(d8 * 2 * (size_t)L * L);
        S.shift2 = c.take(d8 * 2);
        for (size_t* f : {&S.G1, &S.G2}) *f = c.take(d8 * 2 * (size_t)L * Lk);
        S.Wv = c.take(d8 * (size_t)L * Lk);
    }
    S.total = c.off;
    return true;
}

rsvd_status sp_workspace_bytes(const rsvd_matrix* A, const rsvd_params* p, size_t* bytes) {
    rsvd_status st = check_single_pass(A, p);
    if (st != RSVD_OK) return st;
    SpLayout S;
    if (!sp_layout(A->dtype, p->algorithm, A->rows, A->cols, p->k, p->p, S)) return RSVD_ERR_UNSUPPORTED;
    *bytes = S.total;
    return RSVD_OK;
}

// Small SVD of B (l x L valid rows x cols of Bt = B^T, FP64, ld ldb):
// Gram, shifted Cholesky, one-sided Jacobi, as in Algorithm 4 step 7.
rsvd_status small_svd(rsvd_handle* hp, const Plan& P, void* ws, const double* Bt, int ldb, int rows, int l, int L,
                      double* sigma, double* Ut, double* Mv, int max_sweeps, hipStream_t s) {
    DevFlags* flags = at<DevFlags>(ws, P.flags);
    RSVD_TRY(launch_gram(0, Bt, ldb, rows, L, at<double>(ws, P.GP), nullptr, s));
    RSVD_TRY(launch_chol(at<double>(ws, P.GP), rows, l, L, at<double>(ws, P.R), at<double>(ws, P.Rinv), flags, 2,
                         at<double>(ws, P.shift), at<double>(ws, P.work), 0.0, s));
    rsvd_handle::Rec jac{6, nullptr, nullptr};
    if (hp) {
        jac.start = hp->get_event();
        jac.stop = hp->get_event();
        if (!jac.start || !jac.stop) return RSVD_ERR_DEVICE;
        RSVD_TRY(hipEventRecord(jac.start, s));
    }
    RSVD_TRY(launch_jacobi(at<double>(ws, P.R), l, L, at<double>(ws, P.shift), sigma, Ut, Mv, flags,
                           at<double>(ws, P.work), jacobi_tol(P.dtype), s, max_sweeps));
    if (hp) {
        RSVD_TRY(hipEventRecord(jac.stop, s));
        hp->recs.push_back(jac);
    }
    return RSVD_OK;
}

// Two independent small SVDs of the same size in one Jacobi launch (two
// workgroups): Bt0, Bt1 (rows x L, ld ldb) -> sigma + b L, Ut + b L^2
// (factors R2 + b L^2, shifts shift2[b], Mv scratch Mv2 + b L^2).
rsvd_status small_svd2(rsvd_handle* hp, const Plan& P, void* ws, const double* Bt0, const double* Bt1, int ldb,
                       int rows, int l, int L, double* R2, double* shift2, double* sigma, double* Ut, double* Mv2,
                       int max_sweeps, hipStream_t s) {
    DevFlags* flags = at<DevFlags>(ws, P.flags);
    for (int b = 0; b < 2; ++b) {
        RSVD_TRY(launch_gram(0, b ? Bt1 : Bt0, ldb, rows, L, at<double>(ws, P.GP), nullptr, s));
        RSVD_TRY(launch_chol(at<double>(ws, P.GP), rows, l, L, R2 + (size_t)b * L * L, at<double>(ws, P.Rinv), flags,
                             2, shift2 + b, at<double>(ws, P.work), 0.0, s));
    }
    rsvd_handle::Rec jac{6, nullptr, nullptr};
    if (hp) {
        jac.start = hp->get_event();
        jac.stop = hp->get_event();
        if (!jac.start || !jac.stop) return RSVD_ERR_DEVICE;
        RSVD_TRY(hipEventRecord(jac.start, s));
    }
    RSVD_TRY(launch_jacobi(R2, l, L, shift2, sigma, Ut, Mv2, flags, at<double>(ws, P.work), jacobi_tol(P.dtype), s,
                           max_sweeps, 2));
    if (hp) {
        RSVD_TRY(hipEventRecord(jac.stop, s));
        hp->recs.push_back(jac);
    }
    return RSVD_OK;
}

// U (m x k) = Qu Wu and Vt (k x n) = (Qv Wv)^T with the sign rule of
// Algorithm 4 (largest-magnitude entry of each V column positive); S = vals.
rsvd_status finish_factors(const Plan& P, void* ws, int dt, const void* Qu, int64_t m, const double* Wu,
                           const void* Qv, int64_t n, const double* Wv, int ldw, int k, const double* vals,
                           const rsvd_result* out, hipStream_t s) {
    const int L = P.L;
    double* av = at<double>(ws, P.amax_val);
    int* ai = at<int>(ws, P.amax_idx);
    double* sign = at<double>(ws, P.sign);
    RSVD_TRY(launch_apply(dt, Qv, L, n, L, Wv, ldw, k, out->Vt, out->ldvt, 1, nullptr, nullptr, av, ai, 0, s));
    RSVD_TRY(launch_signs(av, ai, apply_blocks(n), k, vals, out->S, sign, s));
    RSVD_TRY(launch_apply(dt, Qu, L, m, L, Wu, ldw, k, out->U, out->ldu, 0, sign, nullptr, nullptr, nullptr, 0, s));
    RSVD_TRY(launch_scale_rows(dt, out->Vt, out->ldvt, k, n, sign, s));
    return RSVD_OK;
}

rsvd_status solve_single_pass(rsvd_handle* hp, const SpLayout& S, const rsvd_matrix* A, const rsvd_params* params,
                              const rsvd_result* out, void* ws, hipStream_t s) {
    const Plan& P = S.base;
    const int dt = P.dtype, L = P.L, l = (int)P.l, k = (int)P.k, Lk = S.Lk;
    const int64_t m = P.m, n = P.n;
    const size_t es = esize(dt);
    const int om = params->orth, sweeps = params->jacobi_max_sweeps;
    DevFlags* flags = at<DevFlags>(ws, P.flags);
    char* pn = at<char>(ws, S.panel_n);
    void* Q1 = at<char>(ws, P.Q);
    void* Q2 = at<char>(ws, P.W);
    double* xpart = at<double>(ws, S.xpart);
    double* CTc = at<double>(ws, S.CTc);
    double* Mv = at<double>(ws, P.Mv);
    double* Wu = at<double>(ws, S.Wu);
    rsvd_status st;
    RSVD_TRY(launch_init(at<int>(ws, P.counters), P.ncounters, flags, s));
    rsvd_handle::Rec stage1{5, nullptr, nullptr};
    if (hp) {
        stage1.start = hp->get_event();
        stage1.stop = hp->get_event();
        if (!stage1.start || !stage1.stop) return RSVD_ERR_DEVICE;
        RSVD_TRY(hipEventRecord(stage1.start, s));
    }
    if (S.alg == 5) {
        // Steps 1-3: Y = A Omega into [Y | Omega] (the one pass over A), Omega
        // beside it (zero padded), Q = orth(Y).
        if ((st = run_product(hp, P, ws, A, 0, nullptr, 0, params->seed, l, L, P.splits_nn, pn, 2 * L, s)) != RSVD_OK)
            return st;
        RSVD_TRY(launch_copy2d(dt, pn + es * L, 2 * L, n, 0, pn + es * L, 2 * L, L, s));
        RSVD_TRY(launch_omega(dt, params->seed, 0, n, l, pn + es * L, 2 * L, s));
        if ((st = run_orth_cols(P, ws, flags, dt, n, l, L, pn, Q1, om, s, 2 * L)) != RSVD_OK) return st;
        if (hp) {
            RSVD_TRY(hipEventRecord(stage1.stop, s));
            hp->recs.push_back(stage1);
        }
        // Step 4: [Z^T ; W^T] = [Y | Omega]^T Q with Z = Q^T Y, W = Q^T Omega;
        // C^T = X from W^T X = Z^T.
        double* X = at<double>(ws, S.X);
        RSVD_TRY(launch_cross(dt, pn, 2 * L, Q1, L, n, 2 * L, L, xpart, CTc, L, s));
        RSVD_TRY(launch_gj_solve(CTc + (size_t)L * L, CTc, L, l, X, L, flags, s));
        // Step 5: eigendecomposition of (C + C^T) / 2 through the shifted
        // positive definite matrix and the small-SVD chain.
        RSVD_TRY(launch_sym_pack(X, L, l, L, at<double>(ws, P.GP), at<double>(ws, S.shiftE), s));
        RSVD_TRY(launch_chol(at<double>(ws, P.GP), l, l, L, at<double>(ws, P.R), at<double>(ws, P.Rinv), flags, 2,
                             at<double>(ws, P.shift), at<double>(ws, P.work), 0.0, s));
        rsvd_handle::Rec jac{6, nullptr, nullptr};
        if (hp) {
            jac.start = hp->get_event();
            jac.stop = hp->get_event();
            if (!jac.start || !jac.stop) return RSVD_ERR_DEVICE;
            RSVD_TRY(hipEventRecord(jac.start, s));
        }
        RSVD_TRY(launch_jacobi(at<double>(ws, P.R), l, L, at<double>(ws, P.shift), at<double>(ws, P.sigma),
                               at<double>(ws, P.Ut), Mv, flags, at<double>(ws, P.work), jacobi_tol(P.dtype), s,
                               sweeps));
        if (hp) {
            RSVD_TRY(hipEventRecord(jac.stop, s));
            hp->recs.push_back(jac);
        }
        double* lam = at<double>(ws, S.lam);
        RSVD_TRY(launch_eig_finish(at<double>(ws, P.sigma), at<double>(ws, P.Ut), l, L, at<double>(ws, S.shiftE), k,
                                   lam, Wu, Lk, s));
        // Step 6: U = Q U^ (and Vt = U^T), eigenvector signs.
        if ((st = finish_factors(P, ws, dt, Q1, n, Wu, Q1, n, Wu, Lk, k, lam, out, s)) != RSVD_OK) return st;
        if (out->Q) RSVD_TRY(launch_copy2d(dt, Q1, L, n, l, out->Q, out->ldq, l, s));
        RSVD_TRY(launch_export_info(flags, out->info, s, out->jacobi_sweeps));
        return RSVD_OK;
    }

    // Algorithm 6.  Steps 1-2: one read of A gives Y_c = A Omega_c (into
    // [Omega_r | Y_c]) and Y_r = A^T Omega_r (into [Y_r | Omega_c]); the
    // kernel also writes both test matrices beside them.
    char* pm = at<char>(ws, S.panel_m);
    DualArgs a{};
    a.A = A->data; a.lda = A->ld; a.M = m; a.K = n; a.seed = params->seed; a.ncols = l; a.wcols = L;
    a.stream_c = 0; a.stream_r = kOmegaRowStream;
    a.Yc = pm + es * L; a.ldyc = 2 * L;
    a.part_c = at<char>(ws, S.part_c); a.splits = S.splits;
    a.part_r = at<char>(ws, S.part_r);
    a.omega_c_out = pn + es * L; a.ldoc = 2 * L;
    a.omega_r_out = pm; a.ldor = 2 * L;
    if (hp) {
        rsvd_handle::Rec rec{7, hp->get_event(), hp->get_event()};
        if (!rec.start || !rec.stop) return RSVD_ERR_DEVICE;
        RSVD_TRY(hipEventRecord(rec.start, s));
        RSVD_TRY(launch_dual_sketch(dt, a, pn, 2 * L, s, rec.stop));
        hp->recs.push_back(rec);
    } else {
        RSVD_TRY(launch_dual_sketch(dt, a, pn, 2 * L, s));
    }
    // Step 3: Q_1 = orth(Y_c), Q_2 = orth(Y_r); the k dominant left singular
    // vectors are Q_1 U^_c(:, 1:k), Q_2 U^_r(:, 1:k) with U^ from the SVD of
    // T_c = Q_1^T Y_c and T_r = Q_2^T Y_r.
    if ((st = run_orth_cols(P, ws, flags, dt, m, l, L, pm + es * L, Q1, om, s, 2 * L)) != RSVD_OK) return st;
    if ((st = run_orth_cols(P, ws, flags, dt, n, l, L, pn, Q2, om, s, 2 * L)) != RSVD_OK) return st;
    if (hp) {
        RSVD_TRY(hipEventRecord(stage1.stop, s));
        hp->recs.push_back(stage1);
    }
    double* CTr = at<double>(ws, S.CTr);
    double *Ut_c = at<double>(ws, S.Ut_cr), *Ut_r = Ut_c + (size_t)L * L;
    double *UtP = at<double>(ws, S.UtPS), *UtS = UtP + (size_t)Lk * Lk, *UtC = at<double>(ws, S.UtC);
    double *sigP = at<double>(ws, S.sigPS), *sigS = sigP + Lk, *sigC = at<double>(ws, S.sigC);
    double *R2 = at<double>(ws, S.R2), *shift2 = at<double>(ws, S.shift2), *Mv2 = at<double>(ws, S.Mv2);
    double *G1 = at<double>(ws, S.G1), *G2 = at<double>(ws, S.G2);
    double *F = at<double>(ws, S.F), *T1 = at<double>(ws, S.T1), *Cm = at<double>(ws, S.Cm);
    double *T2 = at<double>(ws, S.T2), *Ct = at<double>(ws, S.Ct), *T3 = at<double>(ws, S.T3);
    double *MvC = at<double>(ws, S.MvC), *Wv = at<double>(ws, S.Wv);
    // CTc = [Omega_r | Y_c]^T Q_1 = [K_c^T ; T_c^T], CTr = [Y_r | Omega_c]^T Q_2 = [T_r^T ; K_r^T]
    // with K_c = Q_1^T Omega_r, K_r = Q_2^T Omega_c.
    RSVD_TRY(launch_cross(dt, pm, 2 * L, Q1, L, m, 2 * L, L, xpart, CTc, L, s));
    RSVD_TRY(launch_cross(dt, pn, 2 * L, Q2, L, n, 2 * L, L, xpart, CTr, L, s));
    // SVDs of T_c and T_r, side by side.
    if ((st = small_svd2(hp, P, ws, CTc + (size_t)L * L, CTr, L, l, l, L, R2, shift2, at<double>(ws, S.sig_cr),
                         Ut_c, Mv2, sweeps, s)) != RSVD_OK)
        return st;
    // Step 4.  G1 = CTc U^_c,k = [M1 ; N2^T], G2 = CTr U^_r,k = [N1 ; M2^T] with
    // M1 = Omega_r^T Q_c, N1 = Y_r^T Q_r, M2 = Q_r^T Omega_c, N2 = Q_c^T Y_c.
    RSVD_TRY(launch_small_gemm(2 * L, k, L, CTc, L, 0, Ut_c, L, 0, G1, Lk, 2 * L, Lk, s));
    RSVD_TRY(launch_small_gemm(2 * L, k, L, CTr, L, 0, Ut_r, L, 0, G2, Lk, 2 * L, Lk, s));
    // Normal equations of the joint least-squares problem: P C + C S = F with
    // P = M1^T M1 = UtP diag(sigP^2) UtP^T, S = M2 M2^T = UtS diag(sigS^2) UtS^T
    // (eigendecompositions through the small SVDs of M1, M2^T) and
    // F = M1^T N1 + N2 M2^T = G1^T G2.  C = UtP ((UtP^T F UtS) ./ (sigP_i^2 + sigS_j^2)) UtS^T.
    if ((st = small_svd2(hp, P, ws, G1, G2 + (size_t)L * Lk, Lk, l, k, Lk, R2, shift2, sigP, UtP, Mv2, sweeps, s)) !=
        RSVD_OK)
        return st;
    RSVD_TRY(launch_small_gemm(k, k, 2 * L, G1, Lk, 1, G2, Lk, 0, F, Lk, Lk, Lk, s));
    RSVD_TRY(launch_small_gemm(k, k, k, UtP, Lk, 1, F, Lk, 0, T1, Lk, Lk, Lk, s));
    RSVD_TRY(launch_small_gemm(k, k, k, T1, Lk, 0, UtS, Lk, 0, Cm, Lk, Lk, Lk, s, sigP, sigS));
    RSVD_TRY(launch_small_gemm(k, k, k, UtS, Lk, 0, Cm, Lk, 1, T2, Lk, Lk, Lk, s));
    RSVD_TRY(launch_small_gemm(k, k, k, T2, Lk, 0, UtP, Lk, 1, Ct, Lk, Lk, Lk, s));          // C^T
    // Step 5: SVD of C (Bt = C^T): C = UtC diag(sigC) V^^T, V^ = C^T UtC diag(1/sigC).
    if ((st = small_svd(hp, P, ws, Ct, Lk, k, k, Lk, sigC, UtC, MvC, sweeps, s)) != RSVD_OK) return st;
    // Step 6: U = Q_1 (U^_c,k UtC), V = Q_2 (U^_r,k C^T MvC).
    RSVD_TRY(launch_small_gemm(L, k, k, Ut_c, L, 0, UtC, Lk, 0, Wu, Lk, L, Lk, s));
    RSVD_TRY(launch_small_gemm(k, k, k, Ct, Lk, 0, MvC, Lk, 0, T3, Lk, Lk, Lk, s));
    RSVD_TRY(launch_small_gemm(L, k, k, Ut_r, L, 0, T3, Lk, 0, Wv, Lk, L, Lk, s));
    if ((st = finish_factors(P, ws, dt, Q1, m, Wu, Q2, n, Wv, Lk, k, sigC, out, s)) != RSVD_OK) return st;
    if (out->Q) RSVD_TRY(launch_copy2d(dt, Q1, L, m, l, out->Q, out->ldq, l, s));
    RSVD_TRY(launch_export_info(flags, out->info, s, out->jacobi_sweeps));
    return RSVD_OK;
}

// One solve on `stream` with the workspace ws.  profile: allow the event
// records of rsvd_profile_enable (they may create HIP events).
rsvd_status solve_impl(rsvd_handle* h, const rsvd_matrix* A, const rsvd_params* params, const rsvd_result* out,
                       void* ws, size_t ws_bytes, void* stream, bool profile) {
    if (!h || !out) return RSVD_ERR_INVALID_ARG;
    rsvd_status st = check_matrix(A);
    if (st != RSVD_OK) return st;
    if ((st = check_params(A, params)) != RSVD_OK) return st;
    if (single_pass(params)) {
        if ((st = check_single_pass(A, params)) != RSVD_OK) return st;
        SpLayout S;
        if (!sp_layout(A->dtype, params->algorithm, A->rows, A->cols, params->k, params->p, S))
            return RSVD_ERR_UNSUPPORTED;
        if (!out->U || !out->S || !out->Vt || !out->info) return RSVD_ERR_INVALID_ARG;
        if (out->ldu < params->k || out->ldvt < A->cols) return RSVD_ERR_INVALID_ARG;
        if (out->Q && out->ldq < S.base.l) return RSVD_ERR_INVALID_ARG;
        if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return RSVD_ERR_INVALID_ARG;
        if (ws_bytes < S.total) return RSVD_ERR_WORKSPACE_TOO_SMALL;
        if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_DEVICE;
        return solve_single_pass(profile && h->profiling ? h : nullptr, S, A, params, out, ws, as_stream(stream));
    }
    Plan P;
    if (!make_plan(A->dtype, A->rows, A->cols, params->k, params->p, params->q, params->return_full_l, P,
                   params->residual & 1))
        return RSVD_ERR_UNSUPPORTED;
    if (!out->U || !out->S || !out->Vt || !out->info) return RSVD_ERR_INVALID_ARG;
    if (out->ldu < P.r || out->ldvt < P.n) return RSVD_ERR_INVALID_ARG;
    if (out->Q && out->ldq < P.l) return RSVD_ERR_INVALID_ARG;
    if (params->residual && !out->residual) return RSVD_ERR_INVALID_ARG;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return RSVD_ERR_INVALID_ARG;
    if (ws_bytes < P.total) return RSVD_ERR_WORKSPACE_TOO_SMALL;
    if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_DEVICE;

    hipStream_t s = as_stream(stream);
    const int dt = P.dtype;                 // working precision of the panels
    const bool lowp = is_lowp(A->dtype);
    const rsvd_matrix Am = lowp && A->master ? master_view(A) : *A;   // FP32 A for step 6 and the residual
    const int64_t qeff = P.q + (lowp ? (params->extra_power_pass < 0 ? 1 : params->extra_power_pass) : 0);
    const int L = P.L;
    DevFlags* flags = at<DevFlags>(ws, P.flags);
    int* cnt = at<int>(ws, P.counters);
    void* Y = at<char>(ws, P.Y);
    void* Q = at<char>(ws, P.Q);
    void* W = at<char>(ws, P.W);
    const int om = params->orth;

    RSVD_TRY(launch_init(cnt, P.ncounters, flags, s));
    rsvd_handle* hp = profile && h->profiling ? h : nullptr;   // product timing on
    rsvd_handle::Rec stage1{5, nullptr, nullptr};
    if (hp) {
        stage1.start = h->get_event();
        stage1.stop = h->get_event();
        if (!stage1.start || !stage1.stop) return RSVD_ERR_DEVICE;
        RSVD_TRY(hipEventRecord(stage1.start, s));
    }
    if (A->dtype == RSVD_FP8_E4M3) RSVD_TRY(launch_vec_max(A->col_scale, A->cols, at<float>(ws, P.smax), s));
    const int* srft = nullptr;
    if (params->test_matrix == RSVD_TEST_SRFT) {
        RSVD_TRY(launch_srft_columns(params->seed, P.n, (int)P.l, at<int>(ws, P.cols), s));
        srft = at<int>(ws, P.cols);
    }
    if (params->algorithm == 3) {
        // Algorithm 3 (Section 3.2): Y = A Omega, then q times Z = A^T Y,
        // Y = A Z with no orthonormalisation in between; orth once at the end.
        if ((st = run_gemm(hp, P, ws, A, 0, nullptr, params->seed, Y, s, -1, srft)) != RSVD_OK) return st;
        for (int64_t t = 0; t < qeff; ++t) {
            if ((st = run_gemm(hp, P, ws, A, 1, Y, 0, W, s)) != RSVD_OK) return st;
            if ((st = run_gemm(hp, P, ws, A, 0, W, 0, Y, s)) != RSVD_OK) return st;
        }
        if ((st = run_orth(P, ws, dt, P.m, Y, Q, om, s)) != RSVD_OK) return st;
    } else {
        // Stage 1: steps 1-3, sketch with the generated test matrix, then orth.
        if ((st = run_gemm(hp, P, ws, A, 0, nullptr, params->seed, Y, s, -1, srft)) != RSVD_OK) return st;
        if ((st = run_orth(P, ws, dt, P.m, Y, Q, om, s)) != RSVD_OK) return st;
        // Steps 4-5: q power iterations, each product re-orthonormalised.
        for (int64_t t = 0; t < qeff; ++t) {
            if ((st = run_gemm(hp, P, ws, A, 1, Q, 0, Y, s)) != RSVD_OK) return st;
            if ((st = run_orth(P, ws, dt, P.n, Y, W, om, s)) != RSVD_OK) return st;
            if ((st = run_gemm(hp, P, ws, A, 0, W, 0, Y, s)) != RSVD_OK) return st;
            if ((st = run_orth(P, ws, dt, P.m, Y, Q, om, s)) != RSVD_OK) return st;
        }
    }
    if (hp) {
        RSVD_TRY(hipEventRecord(stage1.stop, s));
        h->recs.push_back(stage1);
    }
    // Stage 2: step 6 as B^T = A^T Q (n x l), with the FP32 copy of a
    // low-precision A when there is one; step 7 small SVD, step 8 lift.
    if ((st = run_gemm(hp, P, ws, &Am, 1, Q, 0, Y, s, lowp && A->master ? 4 : -1)) != RSVD_OK) return st;
    const void* Bt = Y;
    double* R = at<double>(ws, P.R);
    double* sigma = at<double>(ws, P.sigma);
    double* sign = at<double>(ws, P.sign);
    double* Ut = at<double>(ws, P.Ut);
    double* Mv = at<double>(ws, P.Mv);
    double* shift = at<double>(ws, P.shift);
    double* av = at<double>(ws, P.amax_val);
    int* ai = at<int>(ws, P.amax_idx);
    const int r = (int)P.r;
    RSVD_TRY(launch_gram(dt, Bt, L, P.n, L, at<double>(ws, P.GP), nullptr, s));
    RSVD_TRY(launch_chol(at<double>(ws, P.GP), P.n, (int)P.l, L, R, at<double>(ws, P.Rinv), flags, 2, shift,
                         at<double>(ws, P.work), 0.0, s));
    rsvd_handle::Rec jac{6, nullptr, nullptr};
    if (hp) {
        jac.start = h->get_event();
        jac.stop = h->get_event();
        if (!jac.start || !jac.stop) return RSVD_ERR_DEVICE;
        RSVD_TRY(hipEventRecord(jac.start, s));
    }
    RSVD_TRY(launch_jacobi(R, (int)P.l, L, shift, sigma, Ut, Mv, flags, at<double>(ws, P.work), jacobi_tol(P.dtype),
                           s, params->jacobi_max_sweeps));
    if (hp) {
        RSVD_TRY(hipEventRecord(jac.stop, s));
        h->recs.push_back(jac);
    }
    // V = B^T U~ Sigma^{-1}, written transposed into Vt, with column argmax partials.
    RSVD_TRY(launch_apply(dt, Bt, L, P.n, L, Mv, L, r, out->Vt, out->ldvt, 1, nullptr, nullptr, av, ai, 0, s));
    RSVD_TRY(launch_signs(av, ai, apply_blocks(P.n), r, sigma, out->S, sign, s));
    // U = Q U~ (top r columns), signs folded in; then the signs of Vt's rows.
    RSVD_TRY(launch_apply(dt, Q, L, P.m, L, Ut, L, r, out->U, out->ldu, 0, sign, nullptr, nullptr, nullptr, 0, s));
    RSVD_TRY(launch_scale_rows(dt, out->Vt, out->ldvt, r, P.n, sign, s));
    if (out->Q) RSVD_TRY(launch_copy2d(dt, Q, L, P.m, (int)P.l, out->Q, out->ldq, (int)P.l, s));
    if (params->residual & 2)
        RSVD_TRY(launch_residual_fro(dt, Am.data, Am.ld, P.m, P.n, Q, Bt, (int)P.l, L, at<double>(ws, P.res_part),
                                     out->residual, s));
    if (params->residual & 1) {
        const int iters = params->residual_iters ? params->residual_iters : kSpecItersDefault;
        if ((st = run_spectral(P, ws, &Am, Q, params->seed, iters, out->residual, params->residual & 2, s)) != RSVD_OK)
            return st;
    }
    RSVD_TRY(launch_export_info(flags, out->info, s, out->jacobi_sweeps));
    return RSVD_OK;
}

}  // namespace

extern "C" {

rsvd_status rsvd_solve(rsvd_handle* h, const rsvd_matrix* A, const rsvd_params* params, const rsvd_result* out,
                       void* ws, size_t ws_bytes, void* stream) {
    return solve_impl(h, A, params, out, ws, ws_bytes, stream, true);
}

rsvd_status rsvd_solve_noalloc(rsvd_handle* h, const rsvd_matrix* A, const rsvd_params* params,
                               const rsvd_result* out, void* stream) {
    if (!h) return RSVD_ERR_INVALID_ARG;
    size_t need = 0;
    rsvd_status st = rsvd_workspace_size(h, A, params, &need);
    if (st != RSVD_OK) return st;
    if (need > kScratchBytes) return RSVD_ERR_TOO_LARGE;
    void* ws = scratch_ptr(h->device);
    if (!ws) return RSVD_ERR_DEVICE;
    return solve_impl(h, A, params, out, ws, kScratchBytes, stream, false);
}

rsvd_status rsvd_omega(int32_t dtype, uint64_t seed, uint32_t stream_id, int64_t n, int64_t l, void* out, int64_t ld,
                       void* stream) {
    if (dtype != RSVD_F32 && dtype != RSVD_F64) return RSVD_ERR_INVALID_ARG;
    if (n < 0 || l < 0 || (n * l > 0 && (!out || ld < l)) || n > ((int64_t)1 << 33)) return RSVD_ERR_INVALID_ARG;
    RSVD_TRY(launch_omega(dtype, seed, stream_id, n, l, out, ld, as_stream(stream)));
    return RSVD_OK;
}

rsvd_status rsvd_srft_omega(int32_t dtype, uint64_t seed, int64_t n, int64_t l, void* out, int64_t ld, int32_t* cols,
                            void* stream) {
    if (dtype != RSVD_F32 && dtype != RSVD_F64) return RSVD_ERR_INVALID_ARG;
    if (l < 1 || l > kMaxL || n < l || n > ((int64_t)1 << 31) || !out || !cols || ld < l) return RSVD_ERR_INVALID_ARG;
    RSVD_TRY(launch_srft_columns(seed, n, (int)l, cols, as_stream(stream)));
    RSVD_TRY(launch_srft_omega(dtype, seed, n, (int)l, cols, out, ld, as_stream(stream)));
    return RSVD_OK;
}

rsvd_status rsvd_philox_words(uint64_t seed, uint32_t stream_id, const uint32_t* ctr, int64_t count, uint32_t* out,
                              void* stream) {
    if (count < 0 || (count > 0 && (!ctr || !out))) return RSVD_ERR_INVALID_ARG;
    RSVD_TRY(launch_philox_words(seed, stream_id, ctr, count, out, as_stream(stream)));
    return RSVD_OK;
}

}  // extern "C"

namespace {
// Workspace of a single product with a BF16 / FP8 A (rsvd_gemm).
struct LpGemmLayout {
    int L = 0, splits = 1;
    int64_t ldt = 0;
    size_t Xt = 0, tsc = 0, amax = 0, smax = 0, part = 0, total = 0;
};
LpGemmLayout lp_gemm_layout(const rsvd_matrix* A, int trans, int64_t ncols) {
    LpGemmLayout W;
    const int64_t M = trans ? A->cols : A->rows, K = trans ? A->rows : A->cols;
    W.L = (int)round_up(ncols, 16);
    W.ldt = round_up(K, 64);
    Carver c;
    W.Xt = c.take((size_t)lowp_bytes(A->dtype) * (size_t)W.L * (size_t)W.ldt);
    W.tsc = c.take(sizeof(float) * (size_t)W.L);
    W.amax = c.take(sizeof(unsigned) * (size_t)W.L);
    W.smax = c.take(sizeof(float));
    W.part = c.take(sizeof(float) * std::max<size_t>(1, lp_partials_elems(M, K, (int)ncols, &W.splits)));
    W.total = c.off;
    return W;
}
}  // namespace

extern "C" {

rsvd_status rsvd_dual_sketch_workspace_size(const rsvd_matrix* A, int64_t l, size_t* bytes) {
    rsvd_status st = check_matrix(A);
    if (st != RSVD_OK) return st;
    if (!bytes || l < 1) return RSVD_ERR_INVALID_ARG;
    if (A->dtype != RSVD_F32 && A->dtype != RSVD_F64) return RSVD_ERR_UNSUPPORTED;
    if (l > kMaxSingleL) return RSVD_ERR_UNSUPPORTED;
    const int L = (int)round_up(l, 16);
    const int64_t m = A->rows, n = A->cols;
    const int splits = dual_splits(A->dtype, m, n);
    Carver c;
    c.take(esize(A->dtype) * (splits > 1 ? (size_t)splits * m * L : 1));
    c.take(esize(A->dtype) * (size_t)dual_row_tiles(A->dtype, m) * n * L);
    *bytes = c.off;
    return RSVD_OK;
}

rsvd_status rsvd_dual_sketch(rsvd_handle* h, const rsvd_matrix* A, uint64_t seed, int64_t l, void* Yc, int64_t ldyc,
                             void* Yr, int64_t ldyr, void* omega_c, int64_t ldoc, void* omega_r, int64_t ldor,
                             void* ws, size_t ws_bytes, void* stream) {
    if (!h) return RSVD_ERR_INVALID_ARG;
    size_t need = 0;
    rsvd_status st = rsvd_dual_sketch_workspace_size(A, l, &need);
    if (st != RSVD_OK) return st;
    if (!Yc || !Yr || ldyc < l || ldyr < l) return RSVD_ERR_INVALID_ARG;
    if ((omega_c && ldoc < l) || (omega_r && ldor < l)) return RSVD_ERR_INVALID_ARG;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return RSVD_ERR_INVALID_ARG;
    if (ws_bytes < need) return RSVD_ERR_WORKSPACE_TOO_SMALL;
    if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_DEVICE;
    const int L = (int)round_up(l, 16);
    const int64_t m = A->rows, n = A->cols;
    const int splits = dual_splits(A->dtype, m, n);
    Carver c;
    const size_t o_pc = c.take(esize(A->dtype) * (splits > 1 ? (size_t)splits * m * L : 1));
    const size_t o_pr = c.take(esize(A->dtype) * (size_t)dual_row_tiles(A->dtype, m) * n * L);
    DualArgs a{};
    a.A = A->data; a.lda = A->ld; a.M = m; a.K = n; a.seed = seed; a.ncols = (int)l; a.wcols = (int)l;
    a.stream_c = 0; a.stream_r = kOmegaRowStream;
    a.Yc = Yc; a.ldyc = ldyc; a.part_c = at<char>(ws, o_pc); a.splits = splits; a.part_r = at<char>(ws, o_pr);
    a.omega_c_out = omega_c; a.ldoc = ldoc; a.omega_r_out = omega_r; a.ldor = ldor;
    RSVD_TRY(launch_dual_sketch(A->dtype, a, Yr, ldyr, as_stream(stream)));
    return RSVD_OK;
}

rsvd_status rsvd_gemm_workspace_size(const rsvd_matrix* A, int32_t trans, int64_t ncols, size_t* bytes) {
    rsvd_status st = check_matrix(A);
    if (st != RSVD_OK) return st;
    if (!bytes || ncols < 1 || ncols > kMaxL) return RSVD_ERR_INVALID_ARG;
    if (is_lowp(A->dtype)) {
        *bytes = lp_gemm_layout(A, trans, ncols).total;
        return RSVD_OK;
    }
    const int64_t M = trans ? A->cols : A->rows, K = trans ? A->rows : A->cols;
    Carver c;
    c.take(sizeof(int) * (size_t)gemm_row_tiles(A->dtype, M, (int)ncols));
    c.take(sizeof(DevFlags));
    c.take(esize(A->dtype) * std::max<size_t>(1, gemm_partials_elems(A->dtype, M, K, (int)ncols, nullptr)));
    *bytes = c.off;
    return RSVD_OK;
}

rsvd_status rsvd_gemm(rsvd_handle* h, const rsvd_matrix* A, int32_t trans, const void* X, int64_t ldx, uint64_t seed,
                      int64_t ncols, void* Y, int64_t ldy, void* ws, size_t ws_bytes, void* stream) {
    if (!h) return RSVD_ERR_INVALID_ARG;
    size_t need = 0;
    rsvd_status st = rsvd_gemm_workspace_size(A, trans, ncols, &need);
    if (st != RSVD_OK) return st;
    if (trans && !X) return RSVD_ERR_INVALID_ARG;
    if (X && ldx < ncols) return RSVD_ERR_INVALID_ARG;
    if (!Y || ldy < ncols) return RSVD_ERR_INVALID_ARG;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return RSVD_ERR_INVALID_ARG;
    if (ws_bytes < need) return RSVD_ERR_WORKSPACE_TOO_SMALL;
    if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_DEVICE;
    hipStream_t s = as_stream(stream);
    const int64_t M = trans ? A->cols : A->rows, K = trans ? A->rows : A->cols;
    if (is_lowp(A->dtype)) {
        const int fmt = A->dtype;
        const LpGemmLayout W = lp_gemm_layout(A, trans, ncols);
        LpGemmArgs a{};
        a.A = A->data; a.lda = A->ld; a.col_scale = fmt == RSVD_FP8_E4M3 ? A->col_scale : nullptr;
        a.trans = trans; a.M = M; a.K = K; a.seed = seed; a.ncols = (int)ncols; a.wcols = (int)ncols;
        a.Y = static_cast<float*>(Y); a.ldy = ldy; a.partials = at<float>(ws, W.part); a.splits = W.splits;
        a.ldt = W.ldt;
        if (X) {
            RSVD_TRY(launch_lp_operand(fmt, static_cast<const float*>(X), K, (int)ncols, ldx,
                                       (fmt == RSVD_FP8_E4M3 && !trans) ? A->col_scale : nullptr, at<char>(ws, W.Xt),
                                       W.ldt, W.L, at<float>(ws, W.tsc), at<unsigned>(ws, W.amax), s));
            a.Xt = at<char>(ws, W.Xt);
            a.xscale = fmt == RSVD_FP8_E4M3 ? at<float>(ws, W.tsc) : nullptr;
        } else if (fmt == RSVD_FP8_E4M3) {
            RSVD_TRY(launch_vec_max(A->col_scale, A->cols, at<float>(ws, W.smax), s));
            a.omega_scale = at<float>(ws, W.smax);
        }
        RSVD_TRY(launch_lp_gemm(fmt, a, s));
        return RSVD_OK;
    }
    Carver c;
    const size_t o_cnt = c.take(sizeof(int) * (size_t)gemm_row_tiles(A->dtype, M, (int)ncols));
    const size_t o_flags = c.take(sizeof(DevFlags));
    const size_t o_part = c.take(0);
    int splits = 1;
    gemm_partials_elems(A->dtype, M, K, (int)ncols, &splits);
    RSVD_TRY(launch_init(at<int>(ws, o_cnt), gemm_row_tiles(A->dtype, M, (int)ncols), at<DevFlags>(ws, o_flags), s));
    GemmArgs g{};
    g.A = A->data; g.lda = A->ld; g.trans = trans; g.M = M; g.K = K;
    g.X = X; g.ldx = ldx; g.seed = seed; g.ncols = (int)ncols; g.wcols = (int)ncols;
    g.Y = Y; g.ldy = ldy; g.partials = at<char>(ws, o_part); g.splits = splits;
    RSVD_TRY(launch_gemm(A->dtype, g, s));
    return RSVD_OK;
}

rsvd_status rsvd_quantize(int32_t dtype, const float* A, int64_t rows, int64_t cols, int64_t lda, void* out,
                          int64_t ldo, float* col_scale, void* stream) {
    if (!is_lowp(dtype) || !A || !out || rows < 0 || cols < 0 || lda < cols || ldo < cols) return RSVD_ERR_INVALID_ARG;
    if (dtype == RSVD_FP8_E4M3 && !col_scale) return RSVD_ERR_INVALID_ARG;
    RSVD_TRY(launch_quantize(dtype, A, rows, cols, lda, out, ldo, col_scale, as_stream(stream)));
    return RSVD_OK;
}

rsvd_status rsvd_orth_workspace_size(int32_t dtype, int64_t rows, int64_t l, size_t* bytes) {
    if (!bytes || (dtype != RSVD_F32 && dtype != RSVD_F64) || l < 1 || rows < l) return RSVD_ERR_INVALID_ARG;
    Plan P;
    if (!make_plan(dtype, rows, l, l, 0, 0, 0, P)) return RSVD_ERR_UNSUPPORTED;
    *bytes = P.total;
    return RSVD_OK;
}

rsvd_status rsvd_orth(rsvd_handle* h, int32_t dtype, int64_t rows, int64_t l, const void* Y, int64_t ldy, void* Qo,
                      int64_t ldq, int32_t orth_mode, int32_t* info, void* ws, size_t ws_bytes, void* stream) {
    if (!h || !Y || !Qo || !info || ldy < l || ldq < l) return RSVD_ERR_INVALID_ARG;
    if (orth_mode < RSVD_ORTH_AUTO || orth_mode > RSVD_ORTH_HOUSEHOLDER) return RSVD_ERR_INVALID_ARG;
    size_t need = 0;
    rsvd_status st = rsvd_orth_workspace_size(dtype, rows, l, &need);
    if (st != RSVD_OK) return st;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return RSVD_ERR_INVALID_ARG;
    if (ws_bytes < need) return RSVD_ERR_WORKSPACE_TOO_SMALL;
    if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_DEVICE;
    Plan P;
    make_plan(dtype, rows, l, l, 0, 0, 0, P);
    hipStream_t s = as_stream(stream);
    DevFlags* flags = at<DevFlags>(ws, P.flags);
    RSVD_TRY(launch_init(at<int>(ws, P.counters), P.ncounters, flags, s));
    void* Yi = at<char>(ws, P.Y);
    void* Qi = at<char>(ws, P.Q);
    RSVD_TRY(launch_copy2d(dtype, Y, ldy, rows, (int)l, Yi, P.L, P.L, s));
    if ((st = run_orth(P, ws, dtype, rows, Yi, Qi, orth_mode, s)) != RSVD_OK) return st;
    RSVD_TRY(launch_copy2d(dtype, Qi, P.L, rows, (int)l, Qo, ldq, (int)l, s));
    RSVD_TRY(launch_export_info(flags, info, s));
    return RSVD_OK;
}

}  // extern "C"

// ---- canonical angles (Section 4.3, Theorem 5) and the adaptive range finder ----
namespace {

// Workspace of rsvd_canonical_sines: the panel [U2 | U1] (rows x (L2 + K1)),
// Gram partials of it, the projection coefficients, and the small-SVD
// buffers of the K1-column residual.
struct SinesLayout {
    int K1 = 0, L2 = 0, LW = 0;
    size_t flags = 0, panel = 0, GP = 0, M = 0, R = 0, Rinv = 0, Ut = 0, Mv = 0, sigma = 0, shift = 0, work = 0,
           total = 0;
};

SinesLayout sines_layout(int dtype, int64_t rows, int64_t k, int64_t l) {
    SinesLayout W;
    W.K1 = (int)round_up(k, 16);
    W.L2 = (int)round_up(l, 16);
    W.LW = W.L2 + W.K1;
    Carver c;
    W.flags = c.take(sizeof(DevFlags));
    W.panel = c.take(esize(dtype) * (size_t)rows * W.LW);
    W.GP = c.take(sizeof(double) * gram_partials_elems(rows, W.LW));
    W.M = c.take(sizeof(double) * (size_t)W.LW * W.K1);
    W.R = c.take(sizeof(double) * (size_t)W.K1 * W.K1);
    W.Rinv = c.take(sizeof(double) * (size_t)W.K1 * W.K1);
    W.Ut = c.take(sizeof(double) * (size_t)W.K1 * W.K1);
    W.Mv = c.take(sizeof(double) * (size_t)W.K1 * W.K1);
    W.sigma = c.take(sizeof(double) * (size_t)W.K1);
    W.shift = c.take(sizeof(double));
    W.work = c.take(sizeof(double) * kJacobiWorkDoubles);
    W.total = c.off;
    return W;
}

// The projection of the block at column `off` of the panel (K1 wide)
// against the panel's first Lq columns, in place: Y <- Y - Q (Q^T Y) with
// the coefficients from the FP64 Gram of [Q | Y].
rsvd_status project_block(int dtype, void* panel, int64_t ldp, int64_t rows, int Lq, int B, int b, double* GP,
                          double* M, hipStream_t s) {
    if (Lq == 0) return RSVD_OK;
    RSVD_TRY(launch_gram(dtype, panel, ldp, rows, Lq + B, GP, nullptr, s));
    RSVD_TRY(launch_proj_coef_w(GP, rows, Lq, B, b, M, s));
    void* out = static_cast<char*>(panel) + esize(dtype) * (size_t)Lq;
    RSVD_TRY(launch_apply(dtype, panel, ldp, rows, Lq + B, M, B, B, out, ldp, 0, nullptr, nullptr, nullptr, nullptr, 0,
                          s));
    return RSVD_OK;
}

}  // namespace

extern "C" {

rsvd_status rsvd_canonical_sines_workspace_size(int32_t dtype, int64_t rows, int64_t k, int64_t l, size_t* bytes) {
    if (!bytes || (dtype != RSVD_F32 && dtype != RSVD_F64) || k < 1 || l < k || rows < l) return RSVD_ERR_INVALID_ARG;
    if (round_up(k, 16) + round_up(l, 16) > kMaxL) return RSVD_ERR_UNSUPPORTED;
    *bytes = sines_layout(dtype, rows, k, l).total;
    return RSVD_OK;
}

rsvd_status rsvd_canonical_sines(rsvd_handle* h, int32_t dtype, int64_t rows, int64_t k, const void* U1, int64_t ld1,
                                 int64_t l, const void* U2, int64_t ld2, double* sines, void* ws, size_t ws_bytes,
                                 void* stream) {
    if (!h || !U1 || !U2 || !sines || ld1 < k || ld2 < l) return RSVD_ERR_INVALID_ARG;
    size_t need = 0;
    rsvd_status st = rsvd_canonical_sines_workspace_size(dtype, rows, k, l, &need);
    if (st != RSVD_OK) return st;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return RSVD_ERR_INVALID_ARG;
    if (ws_bytes < need) return RSVD_ERR_WORKSPACE_TOO_SMALL;
    if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_DEVICE;
    const SinesLayout W = sines_layout(dtype, rows, k, l);
    hipStream_t s = as_stream(stream);
    DevFlags* flags = at<DevFlags>(ws, W.flags);
    char* panel = at<char>(ws, W.panel);
    double* GP = at<double>(ws, W.GP);
    double* M = at<double>(ws, W.M);
    RSVD_TRY(launch_init(nullptr, 0, flags, s));
    RSVD_TRY(launch_copy2d(dtype, U2, ld2, rows, (int)l, panel, W.LW, W.L2, s));
    RSVD_TRY(launch_copy2d(dtype, U1, ld1, rows, (int)k, panel + esize(dtype) * W.L2, W.LW, W.K1, s));
    // E = (I - U2 U2^T) U1, projected twice, in place of U1 in the panel.
    for (int pass = 0; pass < 2; ++pass)
        if ((st = project_block(dtype, panel, W.LW, rows, W.L2, W.K1, (int)k, GP, M, s)) != RSVD_OK) return st;
    // Singular values of E: FP64 Gram, Cholesky (shifted when E is singular), Jacobi.
    const void* E = panel + esize(dtype) * W.L2;
    RSVD_TRY(launch_gram(dtype, E, W.LW, rows, W.K1, GP, nullptr, s));
    RSVD_TRY(launch_chol(GP, rows, (int)k, W.K1, at<double>(ws, W.R), at<double>(ws, W.Rinv), flags, 2,
                         at<double>(ws, W.shift), at<double>(ws, W.work), 0.0, s));
    RSVD_TRY(launch_jacobi(at<double>(ws, W.R), (int)k, W.K1, at<double>(ws, W.shift), at<double>(ws, W.sigma),
                           at<double>(ws, W.Ut), at<double>(ws, W.Mv), flags, at<double>(ws, W.work), kJacobiTolF64,
                           s));
    RSVD_TRY(launch_sines(at<double>(ws, W.sigma), (int)k, sines, s));
    return RSVD_OK;
}

}  // extern "C"

namespace {

constexpr uint32_t kAdaptiveStream = 3;
constexpr double kEstFactor = 7.978845608028654;    // 10 sqrt(2 / pi)

// Workspace of rsvd_adaptive_range: the orth plan of one block (B columns),
// the panel [Q | block] (rows x PW, PW = round16(max_l) + B), the wide Gram
// partials and projection coefficients, a block buffer and the statistics.
struct AdaptLayout {
    int B = 0, PW = 0;
    Plan orth;
    int splits = 1;
    size_t orth_bytes = 0, part = 0, panel = 0, GP = 0, M = 0, T = 0, T2 = 0, stats = 0, total = 0;
};

AdaptLayout adapt_layout(int dtype, int64_t rows, int64_t cols, int b, int max_l) {
    AdaptLayout W;
    W.B = (int)round_up(b, 16);
    W.PW = (int)round_up(max_l, 16) + W.B;
    make_plan(dtype, rows, W.B, W.B, 0, 0, 0, W.orth);
    Carver c;
    W.orth_bytes = c.take(W.orth.total);
    W.part = c.take(esize(dtype) * std::max<size_t>(1, gemm_partials_elems(dtype, rows, cols, W.B, &W.splits)));
    W.panel = c.take(esize(dtype) * (size_t)rows * W.PW);
    W.GP = c.take(sizeof(double) * gram_partials_elems(rows, W.PW));
    W.M = c.take(sizeof(double) * (size_t)W.PW * W.B);
    W.T = c.take(esize(dtype) * (size_t)rows * W.B);
    W.T2 = c.take(esize(dtype) * (size_t)rows * W.B);
    W.stats = c.take(sizeof(double) * 2);
    W.total = c.off;
    return W;
}

}  // namespace

extern "C" {

rsvd_status rsvd_adaptive_range_workspace_size(const rsvd_matrix* A, int32_t block, int64_t max_l, size_t* bytes) {
    rsvd_status st = check_matrix(A);
    if (st != RSVD_OK) return st;
    if (!bytes || block < 1 || block > 32 || max_l < 1) return RSVD_ERR_INVALID_ARG;
    if (A->dtype != RSVD_F32 && A->dtype != RSVD_F64) return RSVD_ERR_UNSUPPORTED;
    const int64_t cap = std::min<int64_t>(max_l, std::min(A->rows, A->cols));
    if (round_up(cap, 16) + round_up(block, 16) > kMaxL) return RSVD_ERR_UNSUPPORTED;
    *bytes = adapt_layout(A->dtype, A->rows, A->cols, block, (int)cap).total;
    return RSVD_OK;
}

rsvd_status rsvd_adaptive_range(rsvd_handle* h, const rsvd_matrix* A, double tol, int32_t block, int64_t max_l,
                                uint64_t seed, void* Q, int64_t ldq, int64_t* l_out, double* est_out,
                                int32_t* converged_out, void* ws, size_t ws_bytes, void* stream) {
    if (!h || !Q || !l_out || !est_out || !converged_out || !(tol >= 0.0)) return RSVD_ERR_INVALID_ARG;
    size_t need = 0;
    rsvd_status st = rsvd_adaptive_range_workspace_size(A, block, max_l, &need);
    if (st != RSVD_OK) return st;
    const int64_t m = A->rows, n = A->cols;
    const int cap = (int)std::min<int64_t>(max_l, std::min(m, n));
    if (ldq < cap) return RSVD_ERR_INVALID_ARG;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return RSVD_ERR_INVALID_ARG;
    if (ws_bytes < need) return RSVD_ERR_WORKSPACE_TOO_SMALL;
    if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_DEVICE;
    const int dt = A->dtype;
    const size_t es = esize(dt);
    const AdaptLayout W = adapt_layout(dt, m, n, block, cap);
    const Plan& OP = W.orth;
    void* ows = at<char>(ws, W.orth_bytes);           // the orth plan's own region
    char* panel = at<char>(ws, W.panel);
    double* GP = at<double>(ws, W.GP);
    double* M = at<double>(ws, W.M);
    char* T = at<char>(ws, W.T);
    char* T2 = at<char>(ws, W.T2);
    double* dstats = at<double>(ws, W.stats);
    DevFlags* flags = at<DevFlags>(ows, OP.flags);
    hipStream_t s = as_stream(stream);
    const int B = W.B, b = block;
    const double thr = tol / kEstFactor;
    RSVD_TRY(launch_init(at<int>(ows, OP.counters), OP.ncounters, flags, s));
    int lc = 0;                                         // columns of Q so far
    double est = 0.0;
    int converged = 0;
    for (int64_t t = 0;; ++t) {
        const int Lq = (int)round_up(lc, 16);
        char* Yb = panel + es * (size_t)Lq;
        // Y = A Omega_t (columns t b .. t b + b - 1 of the stream-3 test matrix), B wide, zero padded.
        GemmArgs g{};
        g.A = A->data; g.lda = A->ld; g.trans = 0; g.M = m; g.K = n; g.X = nullptr; g.ldx = 0; g.seed = seed;
        g.ncols = b; g.wcols = B; g.Y = Yb; g.ldy = W.PW; g.partials = at<char>(ws, W.part);
        g.splits = W.splits;
        g.omega_stream = kAdaptiveStream;
        g.omega_col0 = t * b;
        RSVD_TRY(launch_gemm(dt, g, s));
        for (int pass = 0; pass < 2; ++pass)
            if ((st = project_block(dt, panel, W.PW, m, Lq, B, b, GP, M, s)) != RSVD_OK) return st;
        // Column norms and the singular values of the projected block.
        RSVD_TRY(launch_gram(dt, Yb, W.PW, m, B, GP, nullptr, s));
        RSVD_TRY(launch_chol(GP, m, b, B, at<double>(ows, OP.R), at<double>(ows, OP.Rinv), flags, 2,
                             at<double>(ows, OP.shift), at<double>(ows, OP.work), 0.0, s));
        RSVD_TRY(launch_jacobi(at<double>(ows, OP.R), b, B, at<double>(ows, OP.shift), at<double>(ows, OP.sigma),
                               at<double>(ows, OP.Ut), at<double>(ows, OP.Mv), flags, at<double>(ows, OP.work),
                               kJacobiTolF64, s));
        RSVD_TRY(launch_adaptive_stats(GP, m, B, b, at<double>(ows, OP.sigma), kEstFactor, thr, dstats, s));
        double hst[2] = {0.0, 0.0};
        RSVD_TRY(hipMemcpyAsync(hst, dstats, sizeof(hst), hipMemcpyDeviceToHost, s));
        RSVD_TRY(hipStreamSynchronize(s));
        est = hst[0];
        const int keep = (int)hst[1];
        if (est <= tol) { converged = 1; break; }
        if (keep < 1 || lc + keep > cap) break;
        // W = Y Z_keep S_keep^-1 (the kept left singular vectors), projected against Q once more, orthonormalised.
        const int Kp = (int)round_up(keep, 16);
        RSVD_TRY(launch_apply(dt, Yb, W.PW, m, B, at<double>(ows, OP.Mv), B, keep, T, B, 0, nullptr, nullptr, nullptr,
                              nullptr, 0, s));
        RSVD_TRY(launch_copy2d(dt, T, B, m, keep, Yb, W.PW, Kp, s));
        if ((st = project_block(dt, panel, W.PW, m, Lq, Kp, keep, GP, M, s)) != RSVD_OK) return st;
        RSVD_TRY(launch_copy2d(dt, Yb, W.PW, m, keep, T, Kp, Kp, s));
        if ((st = run_orth_cols(OP, ows, flags, dt, m, keep, Kp, T, T2, RSVD_ORTH_AUTO, s)) != RSVD_OK) return st;
        // Append: the new columns go right after the last one of Q, zero padding after them.
        RSVD_TRY(launch_copy2d(dt, T2, Kp, m, keep, panel + es * (size_t)lc, W.PW,
                               (int)round_up(lc + keep, 16) - lc, s));
        lc += keep;
    }
    if (lc > 0) RSVD_TRY(launch_copy2d(dt, panel, W.PW, m, lc, Q, ldq, lc, s));
    RSVD_TRY(hipStreamSynchronize(s));
    *l_out = lc;
    *est_out = est;
    *converged_out = converged;
    return RSVD_OK;
}
}  // extern "C"
