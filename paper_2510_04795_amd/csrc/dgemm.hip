// Native FP64 GEMM on the FP64 matrix cores (v_mfma_f64_16x16x4_f64): the
// comparator for the emulated path and the slices = 0 mode of every entry
// point.  Any summation order is a valid FP64 GEMM, so this path is checked
// against the textbook gamma_K |A||B| bound, not bit for bit.
//
// Operand layout of the 16x16x4 instruction (measured): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register r of lane l
// holds C[4 r + l / 16][l % 16].
//
// Tile: 256 threads = 2 x 2 waves of BM/2 x BM/2 outputs in blocks of 16 x 16;
// BM = 128 (each wave 4 x 4 blocks, 64 FP64 accumulators per lane) for large
// problems and the grouped H_eff phases, BM = 64 when the 128 tiles would
// not give every compute unit two workgroups.  K advances 16 at a time
// through two LDS buffers: the next step's operands are loaded into
// registers while the current step is multiplied, then stored to the other
// buffer, one barrier per step.  LDS rows are k-major and padded by four
// doubles so the four k rows a wave reads at once fall in different banks;
// the thread layout of the staging keeps the LDS stores conflict free.
#include "internal.h"

namespace oz {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kBK = 16;

// Tile geometry for a BM x BM tile.
template <int BM>
struct Geo {
    static constexpr int LD = BM + 4;            // padded LDS row (doubles): the 4 k rows a wave reads shift banks
    static constexpr int PER = BM * kBK / 256;   // doubles per thread per operand and K step
    static constexpr int NB = BM / 32;           // 16 x 16 blocks per wave and dimension
    static constexpr int LDS = 4 * kBK * LD;     // two buffers of A and B
};

// Global -> register staging of one K step.  Two thread layouts, chosen by
// which dimension of the stored operand is contiguous:
//   along K  (op(A) = A, op(B) = B^T): thread t takes PER consecutive k of
//            row t % BM; the LDS stores of a wave then cover 64 consecutive
//            rows of one k row (no bank conflicts);
//   across K (op(A) = A^T, op(B) = B): thread t takes PER consecutive rows /
//            columns ((t % 16) PER) of k row t / 16: contiguous runs.
// LDS holds both operands k-major: s[k][row] with rows padded to LD.
template <int PER>
__device__ __forceinline__ void fetch_run(double (&r)[PER], const double *p, bool full, int valid) {
    if (full) {
#pragma unroll
        for (int q = 0; q < PER; q += 2) {
            double2 v;
            __builtin_memcpy(&v, p + q, sizeof(v));
            r[q] = v.x;
            r[q + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < PER; ++q) r[q] = q < valid ? p[q] : 0.0;
    }
}

// rows x K operand stored with K contiguous (row i, k at X[i * ld + k])
template <int BM>
__device__ __forceinline__ void fetch_along_k(double (&r)[Geo<BM>::PER], const double *X, int64_t ld, int rows,
                                              int K, int r0, int k0) {
    constexpr int PER = Geo<BM>::PER;
    const int t = threadIdx.x;
    const int i = r0 + t % BM, k = k0 + (t / BM) * PER;
    const int valid = i < rows ? (K - k < PER ? K - k : PER) : 0;
    fetch_run<PER>(r, X + static_cast<int64_t>(i < rows ? i : 0) * ld + (valid > 0 ? k : 0), valid == PER, valid);
}

template <int BM>
__device__ __forceinline__ void store_along_k(const double (&r)[Geo<BM>::PER], double *s) {
    constexpr int PER = Geo<BM>::PER;
    const int t = threadIdx.x;
    const int i = t % BM, k = (t / BM) * PER;
#pragma unroll
    for (int q = 0; q < PER; ++q) s[(k + q) * Geo<BM>::LD + i] = r[q];
}

// K x cols operand stored with cols contiguous (k, col j at X[k * ld + j])
template <int BM>
__device__ __forceinline__ void fetch_across_k(double (&r)[Geo<BM>::PER], const double *X, int64_t ld, int cols,
                                               int K, int c0, int k0) {
    constexpr int PER = Geo<BM>::PER;
    const int t = threadIdx.x;
    const int k = k0 + (t >> 4), j = c0 + (t & 15) * PER;
    const int valid = k < K ? (cols - j < PER ? cols - j : PER) : 0;
    fetch_run<PER>(r, X + static_cast<int64_t>(k < K ? k : 0) * ld + (valid > 0 ? j : 0), valid == PER, valid);
}

template <int BM>
__device__ __forceinline__ void store_across_k(const double (&r)[Geo<BM>::PER], double *s) {
    constexpr int PER = Geo<BM>::PER;
    const int t = threadIdx.x;
    const int k = t >> 4, j = (t & 15) * PER;
#pragma unroll
    for (int q = 0; q < PER; ++q) s[k * Geo<BM>::LD + j + q] = r[q];
}

template <int BM, bool TA>
__device__ __forceinline__ void fetch_a(double (&ra)[Geo<BM>::PER], const double *A, int64_t lda, int M, int K,
                                        int m0, int k0) {
    if (!TA) fetch_along_k<BM>(ra, A, lda, M, K, m0, k0);
    else fetch_across_k<BM>(ra, A, lda, M, K, m0, k0);
}

template <int BM, bool TA>
__device__ __forceinline__ void store_a(const double (&ra)[Geo<BM>::PER], double *sA) {
    if (!TA) store_along_k<BM>(ra, sA);
    else store_across_k<BM>(ra, sA);
}

template <int BM, bool TB>
__device__ __forceinline__ void fetch_b(double (&rb)[Geo<BM>::PER], const double *B, int64_t ldb, int N, int K,
                                        int n0, int k0) {
    if (TB) fetch_along_k<BM>(rb, B, ldb, N, K, n0, k0);
    else fetch_across_k<BM>(rb, B, ldb, N, K, n0, k0);
}

template <int BM, bool TB>
__device__ __forceinline__ void store_b(const double (&rb)[Geo<BM>::PER], double *sB) {
    if (TB) store_along_k<BM>(rb, sB);
    else store_across_k<BM>(rb, sB);
}

template <int BM, bool TA, bool TB, int MODE, typename GetTerm>
__device__ __forceinline__ void dgemm_tile(const Dgemm64Args &a, GetTerm get_term, int tb, int te,
                                           const OutDesc &out, int m0, int n0, double *lds) {
    using Gm = Geo<BM>;
    constexpr int LD = Gm::LD, PER = Gm::PER, NB = Gm::NB;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave >> 1;
    const int wn = wave & 1;
    const int lq = lane >> 4;   // 0..3
    const int l16 = lane & 15;
    // buffer b: A at lds + b * 2 kBK LD, B right after it
    constexpr int kBuf = 2 * kBK * LD;

    // Accumulating mode: the tile's output elements hold the running sum,
    // sigma = fma(alpha_t, c_t, sigma) after every term in list order (the
    // block owns its tile, each thread re-reads only what it wrote), so the
    // FP64 rounding is that of separately summed terms without keeping a
    // second register tile.  The sum starts from +0, or from the stored value
    // when the output continues a term list split over launches (out.cont).
    const int tend = (MODE == kModeAccum) ? te : tb + 1;
    if (MODE == kModeAccum && tb == te) {
        if (out.cont) return;  // nothing to add to the stored sum
#pragma unroll
        for (int mb = 0; mb < NB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = m0 + wm * (BM / 2) + mb * 16 + 4 * r + lq;
                    const int j = n0 + wn * (BM / 2) + nb * 16 + l16;
                    if (i < out.M && j < out.N) out.C[static_cast<int64_t>(i) * out.ldc + j] = 0.0;
                }
        return;
    }
    for (int ti = tb; ti < tend; ++ti) {
        const Term64 T = get_term(ti);
        v4d acc[NB][NB];
#pragma unroll
        for (int mb = 0; mb < NB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = v4d{0.0, 0.0, 0.0, 0.0};
        const int K = T.K;
        const int nk = (K + kBK - 1) / kBK;
        double ra[PER], rb[PER];
        if (nk > 0) {
            fetch_a<BM, TA>(ra, T.A, T.lda, out.M, K, m0, 0);
            fetch_b<BM, TB>(rb, T.B, T.ldb, out.N, K, n0, 0);
            __syncthreads();  // the previous term / tile may still read LDS
            store_a<BM, TA>(ra, lds);
            store_b<BM, TB>(rb, lds + kBK * LD);
            __syncthreads();
        }
        for (int ks = 0; ks < nk; ++ks) {
            const int cur = ks & 1;
            if (ks + 1 < nk) {
                fetch_a<BM, TA>(ra, T.A, T.lda, out.M, K, m0, (ks + 1) * kBK);
                fetch_b<BM, TB>(rb, T.B, T.ldb, out.N, K, n0, (ks + 1) * kBK);
            }
            const double *cA = lds + cur * kBuf;
            const double *cB = cA + kBK * LD;
#pragma unroll
            for (int kk = 0; kk < kBK / 4; ++kk) {
                double af[NB], bf[NB];
#pragma unroll
                for (int mb = 0; mb < NB; ++mb) af[mb] = cA[(kk * 4 + lq) * LD + wm * (BM / 2) + mb * 16 + l16];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) bf[nb] = cB[(kk * 4 + lq) * LD + wn * (BM / 2) + nb * 16 + l16];
#pragma unroll
                for (int mb = 0; mb < NB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mb], bf[nb], acc[mb][nb], 0, 0, 0);
            }
            if (ks + 1 < nk) {
                store_a<BM, TA>(ra, lds + (cur ^ 1) * kBuf);
                store_b<BM, TB>(rb, lds + (cur ^ 1) * kBuf + kBK * LD);
            }
            __syncthreads();
        }
        // the output base is opaque to the optimiser here, so the 16 NB^2
        // element addresses are formed per term instead of being hoisted out
        // of the term loop (where they would not fit in registers)
        double *cbase = out.C;
        asm volatile("" : "+s"(cbase));
#pragma unroll
        for (int mb = 0; mb < NB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // one element's read-modify-write at a time in registers
                    __builtin_amdgcn_sched_barrier(0);
                    const int i = m0 + wm * (BM / 2) + mb * 16 + 4 * r + lq;
                    const int j = n0 + wn * (BM / 2) + nb * 16 + l16;
                    if (i >= out.M || j >= out.N) continue;
                    const double c = acc[mb][nb][r];
                    double *p = cbase + static_cast<int64_t>(i) * out.ldc + j;
                    if (MODE == kModeGemm)
                        *p = (a.beta == 0.0) ? T.alpha * c : fma(T.alpha, c, a.beta * *p);
                    else
                        *p = fma(T.alpha, c, (ti == tb && !out.cont) ? 0.0 : *p);
                }
    }
}

// XCD-aware tile order (blocks are dispatched to the 8 XCDs round robin).
__device__ __forceinline__ void tile_order(int b, int tiles_m, int tiles_n, int &tm, int &tn) {
    const int T = tiles_m * tiles_n;
    const int q = T / 8, rem = T - q * 8;
    const int x = b % 8, idx = b / 8;
    const int lin = x * q + (x < rem ? x : rem) + idx;
    const int per_group = 4 * tiles_n;
    const int gid = lin / per_group;
    const int first = gid * 4;
    const int rows = tiles_m - first < 4 ? tiles_m - first : 4;
    const int w = lin - gid * per_group;
    tm = first + w % rows;
    tn = w / rows;
}

template <int BM, bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void k_dgemm_single(Dgemm64Args a, int tiles_m) {
    __shared__ double lds[Geo<BM>::LDS];
    int tm, tn;
    tile_order(blockIdx.x, tiles_m, a.tiles_n, tm, tn);
    const Term64 term = a.term;
    dgemm_tile<BM, TA, TB, kModeGemm>(a, [&](int) { return term; }, 0, 1, a.out, tm * BM, tn * BM, lds);
}

template <int BM, bool TB, int MODE>
__global__ __launch_bounds__(256, 2) void k_dgemm_grouped(Dgemm64Args a) {
    __shared__ double lds[Geo<BM>::LDS];
    const TileDesc td = a.tiles[blockIdx.x];
    if (td.out < 0) return;  // padding of the XCD order
    OutDesc od = a.outs[td.out];
    if (a.out_base) od.C = a.out_base + reinterpret_cast<intptr_t>(od.C);
    const Term64 *terms = a.terms;
    const double *b_base = a.b_base;
    dgemm_tile<BM, false, TB, MODE>(a,
                                            [&](int i) {
                                                Term64 tm = terms[i];
                                                if (b_base) tm.B = b_base + reinterpret_cast<intptr_t>(tm.B);
                                                return tm;
                                            },
                                            td.term_begin, td.term_end, od, td.m0, td.n0, lds);
}

template <int BM>
void launch_single_bm(bool ta, bool tb, Dgemm64Args a, hipStream_t s) {
    const int tiles_m = static_cast<int>(ceil_div(a.out.M, BM));
    a.tiles_n = static_cast<int32_t>(ceil_div(a.out.N, BM));
    const unsigned grid = static_cast<unsigned>(tiles_m) * static_cast<unsigned>(a.tiles_n);
    if (!ta && !tb) hipLaunchKernelGGL((k_dgemm_single<BM, false, false>), dim3(grid), dim3(256), 0, s, a, tiles_m);
    if (!ta && tb) hipLaunchKernelGGL((k_dgemm_single<BM, false, true>), dim3(grid), dim3(256), 0, s, a, tiles_m);
    if (ta && !tb) hipLaunchKernelGGL((k_dgemm_single<BM, true, false>), dim3(grid), dim3(256), 0, s, a, tiles_m);
    if (ta && tb) hipLaunchKernelGGL((k_dgemm_single<BM, true, true>), dim3(grid), dim3(256), 0, s, a, tiles_m);
}

}  // namespace

int dgemm_tile_for(int64_t tiles128, int num_cu) { return tiles128 < 2 * static_cast<int64_t>(num_cu) ? 64 : 128; }

hipError_t launch_dgemm_single(bool ta, bool tb, const Dgemm64Args &a, int num_cu, hipStream_t s) {
    if (a.out.M <= 0 || a.out.N <= 0) return hipSuccess;
    if (dgemm_tile_for(ceil_div(a.out.M, 128) * ceil_div(a.out.N, 128), num_cu) == 64)
        launch_single_bm<64>(ta, tb, a, s);
    else
        launch_single_bm<128>(ta, tb, a, s);
    return hipGetLastError();
}

template <int BM>
void launch_grouped_bm(bool tb, const Dgemm64Args &a, hipStream_t s) {
    const bool acc = a.mode == kModeAccum;
    if (tb && acc) hipLaunchKernelGGL((k_dgemm_grouped<BM, true, kModeAccum>), dim3(a.ntiles), dim3(256), 0, s, a);
    if (tb && !acc) hipLaunchKernelGGL((k_dgemm_grouped<BM, true, kModeGemm>), dim3(a.ntiles), dim3(256), 0, s, a);
    if (!tb && acc) hipLaunchKernelGGL((k_dgemm_grouped<BM, false, kModeAccum>), dim3(a.ntiles), dim3(256), 0, s, a);
    if (!tb && !acc) hipLaunchKernelGGL((k_dgemm_grouped<BM, false, kModeGemm>), dim3(a.ntiles), dim3(256), 0, s, a);
}

hipError_t launch_dgemm_grouped(bool tb, const Dgemm64Args &a, hipStream_t s) {
    if (a.ntiles == 0) return hipSuccess;
    if (a.tile == 64)
        launch_grouped_bm<64>(tb, a, s);
    else if (a.tile == 128)
        launch_grouped_bm<128>(tb, a, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace oz
