// Skinny products with the large matrix A on MFMA (gfx950).
//
// Every pass over A in Algorithm 4 is a product of A (or A^T) with a thin
// matrix of l columns: the sketch Y = A Omega (step 2), the power-loop
// products Z = A^T Q and Y = A W (steps 4-5) and the projection
// B^T = A^T Q (step 6).  These passes are the tau_A (k + p) terms of the cost
// model in Section 3.1.1 and dominate the run time.
//
// Kernel shape.  A workgroup of 4 wavefronts owns BM output rows and all
// L = 16 * LT output columns (the whole thin dimension), and one slice of
// the reduction dimension (split-K, `splits` slices).  Each wavefront owns
// 16 * RT rows and issues 16x16x4 MFMAs over RT x LT accumulator tiles, so
// one LDS fragment of A feeds LT MFMAs and one fragment of X feeds RT.
// A is streamed HBM -> registers -> LDS once per workgroup with 16-byte
// loads, one tile ahead of the MFMAs.  The thin operand comes either from
// device memory or, for the sketch, from the counter-based generator
// evaluated straight into LDS (Omega never touches HBM).
//
// Split-K reduction is deterministic: every slice writes its partial tile
// and a separate kernel sums the slices in slice order.  (Reducing inside
// the product kernel needs a device-scope release/acquire per workgroup; on
// this chip that writes back and invalidates the XCD's L2 and costs more
// than the whole reduction kernel.)  Block ids map slice-fastest, so with 8
// slices each XCD (ids are dealt round-robin over the 8 XCDs) holds one K
// slice of every row tile and reads one slice of the thin operand into its
// own L2.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "philox.hpp"

namespace rsvd {

// ---- product kernel (begin) ----
// Rows per wavefront (16 * RT) and K tile.  Wide thin operands (LT > 9, i.e.
// more than 144 columns) use one row tile per wavefront and a shorter K tile
// to keep the accumulators and the prefetch registers within the register
// file.
template <typename T, int LT> struct GemmTile;
template <int LT> struct GemmTile<float, LT> {
    static constexpr int RT = LT > 9 ? 1 : 2, BK = LT > 9 ? 32 : 64;
};
template <int LT> struct GemmTile<double, LT> { static constexpr int RT = 1, BK = 16; };

template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int n = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int n = 2; };

template <typename T>
__device__ __forceinline__ void vec_store(T* dst, const typename Vec16<T>::type& v) {
    *reinterpret_cast<typename Vec16<T>::type*>(dst) = v;
}
template <typename T>
__device__ __forceinline__ T vget(const typename Vec16<T>::type& v, int i);
template <> __device__ __forceinline__ float vget<float>(const float4& v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}
template <> __device__ __forceinline__ double vget<double>(const double2& v, int i) { return i == 0 ? v.x : v.y; }
template <typename T>
__device__ __forceinline__ void vset(typename Vec16<T>::type& v, int i, T x);
template <> __device__ __forceinline__ void vset<float>(float4& v, int i, float x) {
    if (i == 0) v.x = x; else if (i == 1) v.y = x; else if (i == 2) v.z = x; else v.w = x;
}
template <> __device__ __forceinline__ void vset<double>(double2& v, int i, double x) {
    if (i == 0) v.x = x; else v.y = x;
}

// LDS strides chosen so that the 4 lane groups of an MFMA fragment read hit
// disjoint banks.
template <typename T, int L> struct Strides {
    static constexpr int BK = GemmTile<T, L / 16>::BK;
    static constexpr int BM = 64 * GemmTile<T, L / 16>::RT;
    static constexpr int SA_NN = BK + 16 / (int)sizeof(T);
    static constexpr int SA_TN = BM + 64 / (int)sizeof(T);
    static constexpr int SB = (sizeof(T) == 4) ? ((L % 32 == 16) ? L : L + 16)
                                               : ((L % 32 == 16) ? L + 8 : L + 8);
};

// WAVES wavefronts of 16 RT rows each; the sketch runs 8 (two 4-wavefront
// row tiles under one generated Omega tile: half the generator work per row).
template <typename T, bool TRANS, bool OMEGA, int LT, int WAVES = 4>
__global__ __launch_bounds__(64 * WAVES) void skinny_gemm_kernel(GemmArgs g) {
    static_assert(WAVES == 4 || (WAVES == 8 && !TRANS), "the TN layout is sized for 4 wavefronts");
    constexpr int NT = 64 * WAVES;
    constexpr int RT = GemmTile<T, LT>::RT;
    constexpr int BK = GemmTile<T, LT>::BK;
    constexpr int BM = 16 * RT * WAVES;
    constexpr int L = 16 * LT;
    constexpr int VEC = Vec16<T>::n;
    using V = typename Vec16<T>::type;
    using S = Strides<T, L>;
    constexpr int SA = TRANS ? S::SA_TN : S::SA_NN;
    constexpr int SB = S::SB;
    constexpr int A_ELEMS = TRANS ? BK * SA : BM * SA;
    constexpr int NVA = BM * BK / VEC / NT;                    // A vectors per thread
    constexpr int NVB = (BK * L / VEC + NT - 1) / NT;          // X vectors per thread
    constexpr int NOB = (BK / 4 * L + NT - 1) / NT;            // Omega blocks per thread

    __shared__ __attribute__((aligned(16))) T As[A_ELEMS];
    __shared__ __attribute__((aligned(16))) T Bs[BK * SB];

    const T* __restrict__ A = static_cast<const T*>(g.A);
    const T* __restrict__ X = static_cast<const T*>(g.X);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int splits = g.splits;
    const int split = blockIdx.x % splits;
    const int tile = blockIdx.x / splits;
    const int64_t row0 = (int64_t)tile * BM;
    const int64_t kchunk = round_up(ceil_div(g.K, splits), BK);
    const int64_t kbeg = (int64_t)split * kchunk;
    const int64_t kend = min(g.K, kbeg + kchunk);
    const bool avec = ((g.lda % VEC) == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
    const bool xvec = !OMEGA && ((g.ldx % VEC) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);

    using Acc = typename Acc4<T>::type;
    Acc acc[RT][LT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < LT; ++t) acc[r][t] = Acc{0, 0, 0, 0};

    V ra[NVA];
    V rb[OMEGA ? 1 : NVB];
    T ro[OMEGA ? NOB : 1][4];
    const T srft_sc0 = (T)sqrt(1.0 / (double)g.ncols), srft_sc1 = (T)sqrt(2.0 / (double)g.ncols);

    // Tiles wholly inside A (and the slice) take unguarded 16-byte loads.
    const bool rows_full = avec && (row0 + BM <= g.M);
    auto load_a = [&](int64_t k0) {
        if (rows_full && k0 + BK <= kend) {
#pragma unroll
            for (int it = 0; it < NVA; ++it) {
                const int idx = tid + NT * it;
                int64_t row, col;
                if (!TRANS) { row = row0 + idx / (BK / VEC); col = k0 + (idx % (BK / VEC)) * VEC; }
                else        { row = k0 + idx / (BM / VEC);   col = row0 + (idx % (BM / VEC)) * VEC; }
                ra[it] = *reinterpret_cast<const V*>(A + row * g.lda + col);
            }
            return;
        }
#pragma unroll
        for (int it = 0; it < NVA; ++it) {
            const int idx = tid + NT * it;
            int64_t row, col;                   // element (row, col) of A in memory
            if (!TRANS) { row = row0 + idx / (BK / VEC); col = k0 + (idx % (BK / VEC)) * VEC; }
            else        { row = k0 + idx / (BM / VEC);   col = row0 + (idx % (BM / VEC)) * VEC; }
            const int64_t rlim = TRANS ? kend : g.M;      // rows of A valid here
            const int64_t clim = TRANS ? g.M : kend;      // cols of A valid here
            V v;
            if (row < rlim && avec && col + VEC <= clim) {
                v = *reinterpret_cast<const V*>(A + row * g.lda + col);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    vset<T>(v, e, (row < rlim && col + e < clim) ? A[row * g.lda + col + e] : T(0));
            }
            ra[it] = v;
        }
    };
    auto store_a = [&]() {
#pragma unroll
        for (int it = 0; it < NVA; ++it) {
            const int idx = tid + NT * it;
            if (!TRANS) vec_store<T>(&As[(idx / (BK / VEC)) * SA + (idx % (BK / VEC)) * VEC], ra[it]);
            else        vec_store<T>(&As[(idx / (BM / VEC)) * SA + (idx % (BM / VEC)) * VEC], ra[it]);
        }
    };
    auto load_b = [&](int64_t k0) {
        if constexpr (OMEGA) {
#pragma unroll
            for (int it = 0; it < NOB; ++it) {
                const int idx = tid + NT * it;
                const int gi = idx / L, j = idx % L;
                const int64_t r = k0 + 4 * gi;
                if (idx < BK / 4 * L && j < g.ncols && r < kend) {
                    if (g.omega_kind == kOmegaSrft)
                        srft_block<T>(g.seed, (uint32_t)(r >> 2), g.srft_cols[j], g.K, srft_sc0, srft_sc1, ro[it]);
                    else
                        omega_block<T>(g.seed, g.omega_stream, (uint32_t)(r >> 2), (uint32_t)(g.omega_col0 + j), ro[it]);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (r + e >= kend) ro[it][e] = T(0);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) ro[it][e] = T(0);
                }
            }
        } else {
            if (xvec && g.ncols == L && k0 + BK <= kend) {
#pragma unroll
                for (int it = 0; it < NVB; ++it) {
                    const int idx = tid + NT * it;
                    if (idx < BK * L / VEC) {
                        const int rr = idx / (L / VEC), c = (idx % (L / VEC)) * VEC;
                        rb[it] = *reinterpret_cast<const V*>(X + (k0 + rr) * g.ldx + c);
                    }
                }
                return;
            }
#pragma unroll
            for (int it = 0; it < NVB; ++it) {
                const int idx = tid + NT * it;
                const int rr = idx / (L / VEC), c = (idx % (L / VEC)) * VEC;
                const int64_t r = k0 + rr;
                V v;
                if (idx < BK * L / VEC && r < kend && xvec && c + VEC <= g.ncols) {
                    v = *reinterpret_cast<const V*>(X + r * g.ldx + c);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        vset<T>(v, e, (idx < BK * L / VEC && r < kend && c + e < g.ncols) ? X[r * g.ldx + c + e] : T(0));
                }
                rb[it] = v;
            }
        }
    };
    auto store_b = [&]() {
        if constexpr (OMEGA) {
#pragma unroll
            for (int it = 0; it < NOB; ++it) {
                const int idx = tid + NT * it;
                if (idx < BK / 4 * L) {
                    const int gi = idx / L, j = idx % L;
#pragma unroll
                    for (int e = 0; e < 4; ++e) Bs[(4 * gi + e) * SB + j] = ro[it][e];
                }
            }
        } else {
#pragma unroll
            for (int it = 0; it < NVB; ++it) {
                const int idx = tid + NT * it;
                if (idx < BK * L / VEC) vec_store<T>(&Bs[(idx / (L / VEC)) * SB + (idx % (L / VEC)) * VEC], rb[it]);
            }
        }
    };

    const int wm = wave * 16 * RT;
    const int li = lane & 15, lk = lane >> 4;
    if (kbeg < kend) {
        load_a(kbeg);
        load_b(kbeg);
        for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
            __syncthreads();
            store_a();
            store_b();
            __syncthreads();
            if (k0 + BK < kend) {       // prefetch the next tile while the MFMAs run
                load_a(k0 + BK);
                load_b(k0 + BK);
            }
            // Fragments of k-step s + 1 are read from LDS while the MFMAs of
            // step s issue (two register sets).
            T fa[2][RT], fb[2][LT];
            auto read_frags = [&](int kk, T (&a)[RT], T (&b)[LT]) {
#pragma unroll
                for (int r = 0; r < RT; ++r)
                    a[r] = TRANS ? As[(kk + lk) * SA + wm + 16 * r + li] : As[(wm + 16 * r + li) * SA + kk + lk];
#pragma unroll
                for (int t = 0; t < LT; ++t) b[t] = Bs[(kk + lk) * SB + 16 * t + li];
            };
            read_frags(0, fa[0], fb[0]);
#pragma unroll
            for (int st = 0; st < BK / 4; ++st) {
                const int cur = st & 1;
                if (st + 1 < BK / 4) read_frags(4 * (st + 1), fa[cur ^ 1], fb[cur ^ 1]);
#pragma unroll
                for (int t = 0; t < LT; ++t)
#pragma unroll
                    for (int r = 0; r < RT; ++r) acc[r][t] = mfma16x16x4(fa[cur][r], fb[cur][t], acc[r][t]);
                // Keep that order in the schedule: next step's LDS reads, then this step's MFMAs.
                if (st + 1 < BK / 4) __builtin_amdgcn_sched_group_barrier(0x100, RT + LT, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, RT * LT, 0);
            }
        }
    }

    // Epilogue.
    T* __restrict__ Y = static_cast<T*>(g.Y);
    if (splits == 1) {
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int t = 0; t < LT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = row0 + wm + 16 * r + acc_row<T>(lk, v);
                    const int col = 16 * t + li;
                    if (row < g.M && col < g.wcols) Y[row * g.ldy + col] = acc[r][t][v];
                }
        return;
    }
    T* __restrict__ P = static_cast<T*>(g.partials);
    const int64_t pstride = g.M * L;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < LT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + wm + 16 * r + acc_row<T>(lk, v);
                if (row < g.M) P[split * pstride + row * L + 16 * t + li] = acc[r][t][v];
            }
}
// ---- product kernel (end) ----

// Y = sum of the split-K slices, added in slice order (slice 0 first).
template <typename T, int SMAX>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const T* __restrict__ P, int64_t M, int L, int splits,
                                                            T* __restrict__ Y, int64_t ldy, int wcols) {
    using V = typename Vec16<T>::type;
    constexpr int VEC = Vec16<T>::n;
    const int64_t nvec = M * (L / VEC);
    const int64_t idx = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (idx >= nvec) return;
    const int64_t pstride = M * L;
    V x[SMAX];
#pragma unroll
    for (int sl = 0; sl < SMAX; ++sl)
        if (sl < splits) x[sl] = *reinterpret_cast<const V*>(P + sl * pstride + idx * VEC);
    V sum = x[0];
#pragma unroll
    for (int sl = 1; sl < SMAX; ++sl)
        if (sl < splits)
#pragma unroll
            for (int e = 0; e < VEC; ++e) vset<T>(sum, e, vget<T>(sum, e) + vget<T>(x[sl], e));
    const int64_t row = idx / (L / VEC);
    const int c = (int)(idx % (L / VEC)) * VEC;
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        if (c + e < wcols) Y[row * ldy + c + e] = vget<T>(sum, e);
}

template <typename T, bool TRANS, bool OMEGA>
static hipError_t dispatch_lt(const GemmArgs& a, int LT, dim3 grid, hipStream_t s) {
#define RSVD_LT_CASE(N) \
    case N: hipLaunchKernelGGL((skinny_gemm_kernel<T, TRANS, OMEGA, N>), grid, dim3(256), 0, s, a); break;
    switch (LT) {
        RSVD_LT_CASE(1) RSVD_LT_CASE(2) RSVD_LT_CASE(3) RSVD_LT_CASE(4) RSVD_LT_CASE(5) RSVD_LT_CASE(6)
        RSVD_LT_CASE(7) RSVD_LT_CASE(8) RSVD_LT_CASE(9) RSVD_LT_CASE(10) RSVD_LT_CASE(11) RSVD_LT_CASE(12)
        RSVD_LT_CASE(13) RSVD_LT_CASE(14) RSVD_LT_CASE(15) RSVD_LT_CASE(16) RSVD_LT_CASE(17) RSVD_LT_CASE(18)
        default: return hipErrorInvalidValue;
    }
#undef RSVD_LT_CASE
    return hipGetLastError();
}

// The FP32 sketch with 8 wavefronts (LT <= 8: the registers of wider tiles
// spill at 8 wavefronts).
static hipError_t dispatch_sketch8(const GemmArgs& a, int LT, dim3 grid, hipStream_t s) {
#define RSVD_LT_CASE(N) \
    case N: hipLaunchKernelGGL((skinny_gemm_kernel<float, false, true, N, 8>), grid, dim3(512), 0, s, a); break;
    switch (LT) {
        RSVD_LT_CASE(1) RSVD_LT_CASE(2) RSVD_LT_CASE(3) RSVD_LT_CASE(4) RSVD_LT_CASE(5) RSVD_LT_CASE(6)
        RSVD_LT_CASE(7) RSVD_LT_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef RSVD_LT_CASE
    return hipGetLastError();
}

static int bm_of(int dtype, int LT) {
    return dtype == 0 ? 64 * GemmTile<double, 1>::RT : (LT > 9 ? 64 * GemmTile<float, 10>::RT : 64 * GemmTile<float, 1>::RT);
}
static int bk_of(int dtype, int LT) {
    return dtype == 0 ? GemmTile<double, 1>::BK : (LT > 9 ? GemmTile<float, 10>::BK : GemmTile<float, 1>::BK);
}

int gemm_row_tiles(int dtype, int64_t M, int ncols) {
    return (int)ceil_div(M, bm_of(dtype, (int)ceil_div(ncols, 16)));
}

// Split count: aim for about two workgroups per CU (256 CUs) with at least
// eight K tiles per slice; at most 16 slices.
static int choose_splits(int dtype, int64_t M, int64_t K, int ncols) {
    const int tiles = gemm_row_tiles(dtype, M, ncols);
    const int64_t ktiles = ceil_div(K, bk_of(dtype, (int)ceil_div(ncols, 16)));
    int s = (int)ceil_div(512, tiles);
    s = (int)std::min<int64_t>(s, std::max<int64_t>(1, ktiles / 8));
    s = std::max(1, std::min(s, kMaxSplits));
    if (s > 1 && s < 8 && 8 <= ktiles / 8) s = 8;      // one slice per XCD when it fits
    return s;
}

size_t gemm_partials_elems(int dtype, int64_t M, int64_t K, int ncols, int* splits_out) {
    const int s = choose_splits(dtype, M, K, ncols);
    if (splits_out) *splits_out = s;
    const int L = (int)round_up(ncols, 16);
    return s > 1 ? (size_t)s * (size_t)M * (size_t)L : 0;
}

hipError_t launch_gemm(int dtype, GemmArgs a, hipStream_t s, hipEvent_t product_done) {
    if (a.ncols < 1 || a.ncols > kMaxL || a.M < 0 || a.K < 0) return hipErrorInvalidValue;
    if (a.M == 0) return product_done ? hipEventRecord(product_done, s) : hipSuccess;
    const int LT = (int)ceil_div(a.ncols, 16);
    const bool omega = (a.X == nullptr);
    if (omega && a.trans) return hipErrorInvalidValue;
    if (a.splits < 1 || a.splits > kMaxSplits) return hipErrorInvalidValue;
    dim3 grid(gemm_row_tiles(dtype, a.M, a.ncols) * a.splits);
    // The FP32 sketch up to 128 columns: 8 wavefronts, twice the rows per
    // workgroup (same slices).
    const bool sketch8 = omega && dtype != 0 && LT <= 8;
    const dim3 grid8((unsigned)ceil_div(a.M, 2 * bm_of(dtype, LT)) * a.splits);
    hipError_t e;
    if (dtype == 0) {
        if (a.trans) e = dispatch_lt<double, true, false>(a, LT, grid, s);
        else e = omega ? dispatch_lt<double, false, true>(a, LT, grid, s) : dispatch_lt<double, false, false>(a, LT, grid, s);
    } else {
        if (a.trans) e = dispatch_lt<float, true, false>(a, LT, grid, s);
        else if (sketch8) e = dispatch_sketch8(a, LT, grid8, s);
        else e = omega ? dispatch_lt<float, false, true>(a, LT, grid, s) : dispatch_lt<float, false, false>(a, LT, grid, s);
    }
    if (e == hipSuccess && product_done) e = hipEventRecord(product_done, s);
    if (e != hipSuccess || a.splits == 1) return e;
    const int L = 16 * LT;
    const int64_t nvec = a.M * (L / (dtype == 0 ? 2 : 4));
    dim3 rgrid((unsigned)ceil_div(nvec, 256));
    if (dtype == 0)
        hipLaunchKernelGGL((splitk_reduce_kernel<double, kMaxSplits>), rgrid, dim3(256), 0, s,
                           (const double*)a.partials, a.M, L, a.splits, (double*)a.Y, a.ldy, a.wcols);
    else
        hipLaunchKernelGGL((splitk_reduce_kernel<float, kMaxSplits>), rgrid, dim3(256), 0, s,
                           (const float*)a.partials, a.M, L, a.splits, (float*)a.Y, a.ldy, a.wcols);
    return hipGetLastError();
}

hipError_t launch_splitk_reduce_f32(const float* partials, int64_t M, int L, int splits, float* Y, int64_t ldy,
                                    int wcols, hipStream_t s) {
    const int64_t nvec = M * (L / 4);
    hipLaunchKernelGGL((splitk_reduce_kernel<float, kMaxSplits>), dim3((unsigned)ceil_div(nvec, 256)), dim3(256), 0, s,
                       partials, M, L, splits, Y, ldy, wcols);
    return hipGetLastError();
}

// ---- two-sided sketch of the single-pass Algorithm 6 (begin) ----
// Y_c = A Omega_c (M x l) and Y_r = A^T Omega_r (K x l) from one read of A.
// A workgroup owns BM rows of A and one slice of its K columns, like the
// products above, and keeps the BM x L block of Omega_r in LDS for the whole
// slice.  Each K tile of A is staged once in LDS and feeds both products:
// the A Omega_c MFMAs read it row-wise, the A^T Omega_r MFMAs column-wise.
// The row-dependent XOR-free rotation of each LDS row (dual_swz) makes both
// fragment reads conflict-free.  Y_c accumulates in registers over the
// slice (split-K partials as above); the A^T Omega_r block of a K tile is
// complete over the workgroup's rows only, so it is written as the row
// tile's partial and a second kernel sums the row tiles in order.
template <typename T> struct DualTile;
template <> struct DualTile<float> { static constexpr int BM = 128, BK = 64, SW = 64; };
template <> struct DualTile<double> { static constexpr int BM = 64, BK = 32, SW = 32; };

// Column offset of row r inside an LDS row of SW elements (bank rotation).
// FP32 (64 banks): lanes (li, lk) of a row-wise fragment read rows li,
// columns lk; of a column-wise read rows lk, columns li; both hit 64
// distinct banks.  FP64 (32 two-bank slots): the same for each half-wave.
template <typename T> __device__ __forceinline__ int dual_swz(int r);
template <> __device__ __forceinline__ int dual_swz<float>(int r) { return 16 * (r & 3) + 4 * ((r >> 2) & 3); }
template <> __device__ __forceinline__ int dual_swz<double>(int r) { return 16 * (r & 1) + 2 * ((r >> 1) & 7); }
template <typename T> __device__ __forceinline__ int dual_pos(int r, int c) {
    constexpr int SW = DualTile<T>::SW;
    return r * SW + ((c + dual_swz<T>(r)) & (SW - 1));
}

template <typename T, int L> struct DualStride {
    static constexpr int SB = (sizeof(T) == 4) ? ((L % 32 == 16) ? L : L + 16) : L + 8;
};

template <typename T, int LT>
__global__ __launch_bounds__(256) void dual_sketch_kernel(DualArgs g) {
    using DT = DualTile<T>;
    constexpr int BM = DT::BM, BK = DT::BK;
    constexpr int RT = BM / 64;                      // 16-row tiles per wavefront in A Omega_c
    constexpr int L = 16 * LT;
    constexpr int CT = BK / 16;                      // 16-column tiles per K tile
    constexpr int H = 4 / CT;                        // wavefronts per column tile in A^T Omega_r
    constexpr int LTH = (LT + H - 1) / H;            // l tiles per wavefront in A^T Omega_r
    constexpr int VEC = Vec16<T>::n;
    using V = typename Vec16<T>::type;
    constexpr int SB = DualStride<T, L>::SB;
    constexpr int NVA = BM * BK / VEC / 256;
    constexpr int NOB = (BK / 4 * L + 255) / 256;
    constexpr int NOR = (BM / 4 * L + 255) / 256;

    __shared__ __attribute__((aligned(16))) T As[BM * DT::SW];
    __shared__ __attribute__((aligned(16))) T Bs[BK * SB];     // Omega_c rows of the K tile
    __shared__ __attribute__((aligned(16))) T Os[BM * SB];     // Omega_r rows of the row tile

    const T* __restrict__ A = static_cast<const T*>(g.A);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int splits = g.splits;
    const int split = blockIdx.x % splits;
    const int tile = blockIdx.x / splits;
    const int64_t row0 = (int64_t)tile * BM;
    const int64_t kchunk = round_up(ceil_div(g.K, splits), BK);
    const int64_t kbeg = (int64_t)split * kchunk;
    const int64_t kend = min(g.K, kbeg + kchunk);
    const bool avec = ((g.lda % VEC) == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
    const bool rows_full = avec && (row0 + BM <= g.M);

    // Omega_r rows [row0, row0 + BM) into LDS (zero past M and past l), and
    // into the caller's copy from the first slice.
    T* omr = static_cast<T*>(g.omega_r_out);
#pragma unroll
    for (int it = 0; it < NOR; ++it) {
        const int idx = tid + 256 * it;
        if (idx < BM / 4 * L) {
            const int gi = idx / L, j = idx % L;
            const int64_t r = row0 + 4 * gi;
            T z[4];
            if (j < g.ncols && r < g.M) {
                omega_block<T>(g.seed, g.stream_r, (uint32_t)(r >> 2), (uint32_t)j, z);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (r + e >= g.M) z[e] = T(0);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) z[e] = T(0);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                Os[(4 * gi + e) * SB + j] = z[e];
                if (omr && split == 0 && r + e < g.M && j < g.wcols) omr[(r + e) * g.ldor + j] = z[e];
            }
        }
    }

    using Acc = typename Acc4<T>::type;
    Acc acc[RT][LT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < LT; ++t) acc[r][t] = Acc{0, 0, 0, 0};

    V ra[NVA];
    T ro[NOB][4];
    auto load_a = [&](int64_t k0) {
#pragma unroll
        for (int it = 0; it < NVA; ++it) {
            const int idx = tid + 256 * it;
            const int64_t row = row0 + idx / (BK / VEC), col = k0 + (idx % (BK / VEC)) * VEC;
            if (rows_full && k0 + BK <= kend) {
                ra[it] = *reinterpret_cast<const V*>(A + row * g.lda + col);
                continue;
            }
            V v;
            if (row < g.M && avec && col + VEC <= kend) {
                v = *reinterpret_cast<const V*>(A + row * g.lda + col);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    vset<T>(v, e, (row < g.M && col + e < kend) ? A[row * g.lda + col + e] : T(0));
            }
            ra[it] = v;
        }
    };
    auto load_b = [&](int64_t k0) {
#pragma unroll
        for (int it = 0; it < NOB; ++it) {
            const int idx = tid + 256 * it;
            const int gi = idx / L, j = idx % L;
            const int64_t r = k0 + 4 * gi;
            if (idx < BK / 4 * L && j < g.ncols && r < kend) {
                omega_block<T>(g.seed, g.stream_c, (uint32_t)(r >> 2), (uint32_t)j, ro[it]);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (r + e >= kend) ro[it][e] = T(0);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) ro[it][e] = T(0);
            }
        }
    };
    T* omc = static_cast<T*>(g.omega_c_out);
    auto store_tiles = [&](int64_t k0) {
#pragma unroll
        for (int it = 0; it < NVA; ++it) {
            const int idx = tid + 256 * it;
            const int r = idx / (BK / VEC), c = (idx % (BK / VEC)) * VEC;
            vec_store<T>(&As[dual_pos<T>(r, c)], ra[it]);
        }
#pragma unroll
        for (int it = 0; it < NOB; ++it) {
            const int idx = tid + 256 * it;
            if (idx < BK / 4 * L) {
                const int gi = idx / L, j = idx % L;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    Bs[(4 * gi + e) * SB + j] = ro[it][e];
                    const int64_t r = k0 + 4 * gi + e;
                    if (omc && tile == 0 && r < kend && j < g.wcols) omc[r * g.ldoc + j] = ro[it][e];
                }
            }
        }
    };

    const int wm = wave * 16 * RT;
    const int ct = wave % CT, h = wave / CT;
    T* __restrict__ Pr = static_cast<T*>(g.part_r) + (size_t)tile * (size_t)g.K * L;
    if (kbeg < kend) {
        load_a(kbeg);
        load_b(kbeg);
        for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
            __syncthreads();
            store_tiles(k0);
            __syncthreads();
            if (k0 + BK < kend) {
                load_a(k0 + BK);
                load_b(k0 + BK);
            }
            // Y_c += A(tile rows, K tile) Omega_c(K tile): row-wise fragments.
            {
                T fa[2][RT], fb[2][LT];
                auto frags = [&](int kk, T (&a)[RT], T (&b)[LT]) {
#pragma unroll
                    for (int r = 0; r < RT; ++r) a[r] = As[dual_pos<T>(wm + 16 * r + li, kk + lk)];
#pragma unroll
                    for (int t = 0; t < LT; ++t) b[t] = Bs[(kk + lk) * SB + 16 * t + li];
                };
                frags(0, fa[0], fb[0]);
#pragma unroll
                for (int st = 0; st < BK / 4; ++st) {
                    const int cur = st & 1;
                    if (st + 1 < BK / 4) frags(4 * (st + 1), fa[cur ^ 1], fb[cur ^ 1]);
#pragma unroll
                    for (int t = 0; t < LT; ++t)
#pragma unroll
                        for (int r = 0; r < RT; ++r) acc[r][t] = mfma16x16x4(fa[cur][r], fb[cur][t], acc[r][t]);
                    if (st + 1 < BK / 4) __builtin_amdgcn_sched_group_barrier(0x100, RT + LT, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, RT * LT, 0);
                }
            }
            // Y_r(K tile) partial = A(tile rows, K tile)^T Omega_r(tile rows):
            // column-wise fragments, contraction over the BM rows.
            {
                Acc accr[LTH];
#pragma unroll
                for (int t = 0; t < LTH; ++t) accr[t] = Acc{0, 0, 0, 0};
                T fa[2], fb[2][LTH];
                auto frags = [&](int kk, T& a, T (&b)[LTH]) {
                    a = As[dual_pos<T>(kk + lk, 16 * ct + li)];
#pragma unroll
                    for (int t = 0; t < LTH; ++t) {
                        const int tt = h * LTH + t;
                        b[t] = tt < LT ? Os[(kk + lk) * SB + 16 * tt + li] : T(0);
                    }
                };
                frags(0, fa[0], fb[0]);
#pragma unroll 8
                for (int st = 0; st < BM / 4; ++st) {
                    const int cur = st & 1;
                    if (st + 1 < BM / 4) frags(4 * (st + 1), fa[cur ^ 1], fb[cur ^ 1]);
#pragma unroll
                    for (int t = 0; t < LTH; ++t) accr[t] = mfma16x16x4(fa[cur], fb[cur][t], accr[t]);
                }
#pragma unroll
                for (int t = 0; t < LTH; ++t) {
                    const int tt = h * LTH + t;
                    if (tt >= LT) continue;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t col = k0 + 16 * ct + acc_row<T>(lk, v);
                        if (col < kend) Pr[col * L + 16 * tt + li] = accr[t][v];
                    }
                }
            }
        }
    }

    // Y_c epilogue, as in the products above.
    if (splits == 1) {
        T* __restrict__ Y = static_cast<T*>(g.Yc);
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int t = 0; t < LT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = row0 + wm + 16 * r + acc_row<T>(lk, v);
                    const int col = 16 * t + li;
                    if (row < g.M && col < g.wcols) Y[row * g.ldyc + col] = acc[r][t][v];
                }
        return;
    }
    T* __restrict__ P = static_cast<T*>(g.part_c);
    const int64_t pstride = g.M * L;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < LT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + wm + 16 * r + acc_row<T>(lk, v);
                if (row < g.M) P[split * pstride + row * L + 16 * t + li] = acc[r][t][v];
            }
}

// Y (rows x wcols, ldy) = sum of `slices` partials of rows x L, in slice
// order.  One thread per 16-byte vector; loads are issued 8 slices at a time.
template <typename T>
__global__ __launch_bounds__(256) void slices_reduce_kernel(const T* __restrict__ P, int64_t rows, int L, int slices,
                                                            T* __restrict__ Y, int64_t ldy, int wcols) {
    using V = typename Vec16<T>::type;
    constexpr int VEC = Vec16<T>::n;
    const int64_t nvec = rows * (L / VEC);
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= nvec) return;
    const int64_t pstride = rows * L;
    V sum;
#pragma unroll
    for (int e = 0; e < VEC; ++e) vset<T>(sum, e, T(0));
    for (int s0 = 0; s0 < slices; s0 += 8) {
        V x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (s0 + u < slices) x[u] = *reinterpret_cast<const V*>(P + (s0 + u) * pstride + idx * VEC);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (s0 + u < slices)
#pragma unroll
                for (int e = 0; e < VEC; ++e) vset<T>(sum, e, vget<T>(sum, e) + vget<T>(x[u], e));
    }
    const int64_t row = idx / (L / VEC);
    const int c = (int)(idx % (L / VEC)) * VEC;
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        if (c + e < wcols) Y[row * ldy + c + e] = vget<T>(sum, e);
}

static int dual_bm(int dtype) { return dtype == 0 ? DualTile<double>::BM : DualTile<float>::BM; }
static int dual_bk(int dtype) { return dtype == 0 ? DualTile<double>::BK : DualTile<float>::BK; }

int dual_row_tiles(int dtype, int64_t M) { return (int)ceil_div(M, dual_bm(dtype)); }

int dual_splits(int dtype, int64_t M, int64_t K) {
    const int tiles = dual_row_tiles(dtype, M);
    const int64_t ktiles = ceil_div(K, dual_bk(dtype));
    int s = (int)ceil_div(512, tiles);
    s = (int)std::min<int64_t>(s, std::max<int64_t>(1, ktiles / 4));
    s = std::max(1, std::min(s, kMaxSplits));
    if (s > 1 && s < 8 && 8 <= ktiles / 4) s = 8;
    return s;
}

hipError_t launch_dual_sketch(int dtype, DualArgs a, void* Yr, int64_t ldyr, hipStream_t s, hipEvent_t product_done) {
    if (a.ncols < 1 || a.ncols > kMaxDualL || a.M < 1 || a.K < 1) return hipErrorInvalidValue;
    if (a.splits < 1 || a.splits > kMaxSplits) return hipErrorInvalidValue;
    const int LT = (int)ceil_div(a.ncols, 16);
    const int tiles = dual_row_tiles(dtype, a.M);
    dim3 grid(tiles * a.splits);
#define RSVD_DUAL_CASE(N)                                                                                  \
    case N:                                                                                                \
        if (dtype == 0) hipLaunchKernelGGL((dual_sketch_kernel<double, N>), grid, dim3(256), 0, s, a);     \
        else hipLaunchKernelGGL((dual_sketch_kernel<float, N>), grid, dim3(256), 0, s, a);                 \
        break;
    switch (LT) {
        RSVD_DUAL_CASE(1) RSVD_DUAL_CASE(2) RSVD_DUAL_CASE(3) RSVD_DUAL_CASE(4) RSVD_DUAL_CASE(5)
        RSVD_DUAL_CASE(6) RSVD_DUAL_CASE(7) RSVD_DUAL_CASE(8) RSVD_DUAL_CASE(9)
        default: return hipErrorInvalidValue;
    }
#undef RSVD_DUAL_CASE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (product_done && (e = hipEventRecord(product_done, s)) != hipSuccess) return e;
    const int L = 16 * LT;
    const int vec = dtype == 0 ? 2 : 4;
    if (a.splits > 1) {
        const int64_t nvec = a.M * (L / vec);
        dim3 rgrid((unsigned)ceil_div(nvec, 256));
        if (dtype == 0)
            hipLaunchKernelGGL((splitk_reduce_kernel<double, kMaxSplits>), rgrid, dim3(256), 0, s,
                               (const double*)a.part_c, a.M, L, a.splits, (double*)a.Yc, a.ldyc, a.wcols);
        else
            hipLaunchKernelGGL((splitk_reduce_kernel<float, kMaxSplits>), rgrid, dim3(256), 0, s,
                               (const float*)a.part_c, a.M, L, a.splits, (float*)a.Yc, a.ldyc, a.wcols);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int64_t nvec = a.K * (L / vec);
    dim3 rgrid((unsigned)ceil_div(nvec, 256));
    if (dtype == 0)
        hipLaunchKernelGGL(slices_reduce_kernel<double>, rgrid, dim3(256), 0, s, (const double*)a.part_r, a.K, L,
                           tiles, (double*)Yr, ldyr, a.wcols);
    else
        hipLaunchKernelGGL(slices_reduce_kernel<float>, rgrid, dim3(256), 0, s, (const float*)a.part_r, a.K, L,
                           tiles, (float*)Yr, ldyr, a.wcols);
    return hipGetLastError();
}
// ---- two-sided sketch (end) ----

// ---- SRFT test matrix: sampled columns (Floyd's algorithm) ----
// One wavefront; step t (j = n - l + t) draws x = floor(w (j + 1) / 2^32)
// from word 0 of block (t, 1, 4, 0) and takes x unless an earlier step took
// it, else j.  The membership test is spread over the lanes.
__global__ __launch_bounds__(64) void srft_columns_kernel(uint64_t seed, int64_t n, int l, int* cols) {
    __shared__ int taken[kMaxL];
    const int lane = threadIdx.x;
    for (int t = 0; t < l; ++t) {
        const int64_t j = n - l + t;
        const Philox4 w = philox4x32_10((uint32_t)t, 1u, kSrftStream, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
        const int x = (int)(((uint64_t)w.x[0] * (uint64_t)(j + 1)) >> 32);
        bool dup = false;
        for (int u = lane; u < t; u += 64) dup |= taken[u] == x;
        const bool any = __any(dup);
        const int pick = any ? (int)j : x;
        if (lane == 0) {
            taken[t] = pick;
            cols[t] = pick;
        }
        __syncthreads();
    }
}

hipError_t launch_srft_columns(uint64_t seed, int64_t n, int l, int* cols, hipStream_t s) {
    if (l < 1 || l > kMaxL || n < l || n > ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(srft_columns_kernel, dim3(1), dim3(64), 0, s, seed, n, l, cols);
    return hipGetLastError();
}

template <typename T>
__global__ void srft_omega_kernel(uint64_t seed, int64_t n, int l, const int* cols, T* out, int64_t ld) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t groups = ceil_div(n, 4);
    if (idx >= groups * l) return;
    const int64_t gidx = idx / l;
    const int j = (int)(idx % l);
    const T sc0 = (T)sqrt(1.0 / (double)l), sc1 = (T)sqrt(2.0 / (double)l);
    T z[4];
    srft_block<T>(seed, (uint32_t)gidx, cols[j], n, sc0, sc1, z);
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (4 * gidx + e < n) out[(4 * gidx + e) * ld + j] = z[e];
}

hipError_t launch_srft_omega(int dtype, uint64_t seed, int64_t n, int l, const int* cols, void* out, int64_t ld,
                             hipStream_t s) {
    const int64_t total = ceil_div(n, 4) * l;
    if (total == 0) return hipSuccess;
    dim3 grid((unsigned)ceil_div(total, 256));
    if (dtype == 0)
        hipLaunchKernelGGL(srft_omega_kernel<double>, grid, dim3(256), 0, s, seed, n, l, cols, (double*)out, ld);
    else
        hipLaunchKernelGGL(srft_omega_kernel<float>, grid, dim3(256), 0, s, seed, n, l, cols, (float*)out, ld);
    return hipGetLastError();
}

// ---- test entry points: Omega materialised, raw Philox words ----
template <typename T>
__global__ void omega_kernel(uint64_t seed, uint32_t stream, int64_t n, int64_t l, T* out, int64_t ld) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t groups = ceil_div(n, 4);
    if (idx >= groups * l) return;
    const int64_t gidx = idx / l, j = idx % l;
    T z[4];
    omega_block<T>(seed, stream, (uint32_t)gidx, (uint32_t)j, z);
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (4 * gidx + e < n) out[(4 * gidx + e) * ld + j] = z[e];
}

hipError_t launch_omega(int dtype, uint64_t seed, uint32_t stream, int64_t n, int64_t l, void* out, int64_t ld,
                        hipStream_t s) {
    const int64_t total = ceil_div(n, 4) * l;
    if (total == 0) return hipSuccess;
    dim3 grid((unsigned)ceil_div(total, 256));
    if (dtype == 0) hipLaunchKernelGGL(omega_kernel<double>, grid, dim3(256), 0, s, seed, stream, n, l, (double*)out, ld);
    else hipLaunchKernelGGL(omega_kernel<float>, grid, dim3(256), 0, s, seed, stream, n, l, (float*)out, ld);
    return hipGetLastError();
}

__global__ void philox_words_kernel(uint64_t seed, uint32_t stream, const uint32_t* ctr, int64_t count,
                                    uint32_t* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const Philox4 w = philox4x32_10(ctr[2 * i], ctr[2 * i + 1], stream, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
#pragma unroll
    for (int e = 0; e < 4; ++e) out[4 * i + e] = w.x[e];
}

hipError_t launch_philox_words(uint64_t seed, uint32_t stream, const uint32_t* ctr, int64_t count, uint32_t* out,
                               hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(philox_words_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, s, seed, stream, ctr,
                       count, out);
    return hipGetLastError();
}

}  // namespace rsvd
