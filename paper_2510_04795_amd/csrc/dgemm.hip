// Native FP64 GEMM on the FP64 matrix cores (v_mfma_f64_16x16x4_f64): the
// comparator for the emulated path and the slices = 0 mode of every entry
// point.  Any summation order is a valid FP64 GEMM, so this path is checked
// against the textbook gamma_K |A||B| bound, not bit for bit.
//
// Operand layout of the 16x16x4 instruction (measured): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register r of lane l
// holds C[4 r + l / 16][l % 16].
//
// Tile: 256 threads = 2 x 2 waves, 128 x 128 outputs, each wave 4 x 4 blocks
// of 16 x 16 (64 FP64 accumulators per lane).  K advances 16 at a time
// through two LDS buffers: the next step's operands are loaded into
// registers while the current step is multiplied, then stored to the other
// buffer, one barrier per step.  LDS rows are k-major and padded by four
// doubles so the four k rows a wave reads at once fall in different banks;
// the thread layout of the staging keeps the LDS stores conflict free.
#include "internal.h"

namespace oz {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kBM = 128;
constexpr int kBN = 128;
constexpr int kBK = 16;
constexpr int kLd = kBM + 4;             // padded LDS row (doubles): the 4 k rows a wave reads shift banks
constexpr int kPer = kBM * kBK / 256;    // doubles per thread per operand and K step (8)

// Global -> register staging of one K step.  Two thread layouts, chosen by
// which dimension of the stored operand is contiguous:
//   along K  (op(A) = A, op(B) = B^T): thread t takes 8 consecutive k of
//            row t % 128 (k half t / 128); the LDS stores of a wave then
//            cover 64 consecutive rows of one k row (no bank conflicts);
//   across K (op(A) = A^T, op(B) = B): thread t takes 8 consecutive rows /
//            columns (t % 16) of k row t / 16: contiguous 64-byte runs.
// LDS holds both operands k-major: s[k][row] with rows padded to kLd.
__device__ __forceinline__ void fetch_run(double (&r)[kPer], const double *p, bool full, int valid) {
    if (full) {
#pragma unroll
        for (int q = 0; q < kPer; q += 2) {
            double2 v;
            __builtin_memcpy(&v, p + q, sizeof(v));
            r[q] = v.x;
            r[q + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < kPer; ++q) r[q] = q < valid ? p[q] : 0.0;
    }
}

// rows x K operand stored with K contiguous (row i, k at X[i * ld + k])
__device__ __forceinline__ void fetch_along_k(double (&r)[kPer], const double *X, int64_t ld, int rows, int K,
                                              int r0, int k0) {
    const int t = threadIdx.x;
    const int i = r0 + (t & 127), k = k0 + (t >> 7) * kPer;
    const int valid = i < rows ? (K - k < kPer ? K - k : kPer) : 0;
    fetch_run(r, X + static_cast<int64_t>(i < rows ? i : 0) * ld + (valid > 0 ? k : 0), valid == kPer, valid);
}

__device__ __forceinline__ void store_along_k(const double (&r)[kPer], double *s) {
    const int t = threadIdx.x;
    const int i = t & 127, k = (t >> 7) * kPer;
#pragma unroll
    for (int q = 0; q < kPer; ++q) s[(k + q) * kLd + i] = r[q];
}

// K x cols operand stored with cols contiguous (k, col j at X[k * ld + j])
__device__ __forceinline__ void fetch_across_k(double (&r)[kPer], const double *X, int64_t ld, int cols, int K,
                                               int c0, int k0) {
    const int t = threadIdx.x;
    const int k = k0 + (t >> 4), j = c0 + (t & 15) * kPer;
    const int valid = k < K ? (cols - j < kPer ? cols - j : kPer) : 0;
    fetch_run(r, X + static_cast<int64_t>(k < K ? k : 0) * ld + (valid > 0 ? j : 0), valid == kPer, valid);
}

__device__ __forceinline__ void store_across_k(const double (&r)[kPer], double *s) {
    const int t = threadIdx.x;
    const int k = t >> 4, j = (t & 15) * kPer;
#pragma unroll
    for (int q = 0; q < kPer; ++q) s[k * kLd + j + q] = r[q];
}

template <bool TA>
__device__ __forceinline__ void fetch_a(double (&ra)[kPer], const double *A, int64_t lda, int M, int K,
                                        int m0, int k0) {
    if (!TA) fetch_along_k(ra, A, lda, M, K, m0, k0);
    else fetch_across_k(ra, A, lda, M, K, m0, k0);
}

template <bool TA>
__device__ __forceinline__ void store_a(const double (&ra)[kPer], double *sA) {
    if (!TA) store_along_k(ra, sA);
    else store_across_k(ra, sA);
}

template <bool TB>
__device__ __forceinline__ void fetch_b(double (&rb)[kPer], const double *B, int64_t ldb, int N, int K,
                                        int n0, int k0) {
    if (TB) fetch_along_k(rb, B, ldb, N, K, n0, k0);
    else fetch_across_k(rb, B, ldb, N, K, n0, k0);
}

template <bool TB>
__device__ __forceinline__ void store_b(const double (&rb)[kPer], double *sB) {
    if (TB) store_along_k(rb, sB);
    else store_across_k(rb, sB);
}

template <bool TA, bool TB, int MODE, typename GetTerm>
__device__ __forceinline__ void dgemm_tile(const Dgemm64Args &a, GetTerm get_term, int tb, int te,
                                           const OutDesc &out, int m0, int n0, double *lds) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave >> 1;
    const int wn = wave & 1;
    const int lq = lane >> 4;   // 0..3
    const int l16 = lane & 15;
    // buffer b: A at lds + b * 2 kBK kLd, B right after it
    constexpr int kBuf = 2 * kBK * kLd;

    // accumulated FP64 outputs, only held when summing several terms
    constexpr int SIG = (MODE == kModeAccum) ? 4 : 1;
    double sig[SIG][4][4];
#pragma unroll
    for (int mb = 0; mb < SIG; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) sig[mb][nb][r] = 0.0;

    // only the accumulating mode sums several terms into one tile
    const int tend = (MODE == kModeAccum) ? te : tb + 1;
    for (int ti = tb; ti < tend; ++ti) {
        const Term64 T = get_term(ti);
        v4d acc[4][4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = v4d{0.0, 0.0, 0.0, 0.0};
        const int K = T.K;
        const int nk = (K + kBK - 1) / kBK;
        double ra[kPer], rb[kPer];
        if (nk > 0) {
            fetch_a<TA>(ra, T.A, T.lda, out.M, K, m0, 0);
            fetch_b<TB>(rb, T.B, T.ldb, out.N, K, n0, 0);
            __syncthreads();  // the previous term / tile may still read LDS
            store_a<TA>(ra, lds);
            store_b<TB>(rb, lds + kBK * kLd);
            __syncthreads();
        }
        for (int ks = 0; ks < nk; ++ks) {
            const int cur = ks & 1;
            if (ks + 1 < nk) {
                fetch_a<TA>(ra, T.A, T.lda, out.M, K, m0, (ks + 1) * kBK);
                fetch_b<TB>(rb, T.B, T.ldb, out.N, K, n0, (ks + 1) * kBK);
            }
            const double *cA = lds + cur * kBuf;
            const double *cB = cA + kBK * kLd;
#pragma unroll
            for (int kk = 0; kk < kBK / 4; ++kk) {
                double af[4], bf[4];
#pragma unroll
                for (int mb = 0; mb < 4; ++mb) af[mb] = cA[(kk * 4 + lq) * kLd + wm * 64 + mb * 16 + l16];
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) bf[nb] = cB[(kk * 4 + lq) * kLd + wn * 64 + nb * 16 + l16];
#pragma unroll
                for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb)
                        acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mb], bf[nb], acc[mb][nb], 0, 0, 0);
            }
            if (ks + 1 < nk) {
                store_a<TA>(ra, lds + (cur ^ 1) * kBuf);
                store_b<TB>(rb, lds + (cur ^ 1) * kBuf + kBK * kLd);
            }
            __syncthreads();
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = m0 + wm * 64 + mb * 16 + 4 * r + lq;
                    const int j = n0 + wn * 64 + nb * 16 + l16;
                    const double c = acc[mb][nb][r];
                    if (MODE == kModeGemm) {
                        if (i < out.M && j < out.N) {
                            double *p = out.C + static_cast<int64_t>(i) * out.ldc + j;
                            *p = (a.beta == 0.0) ? T.alpha * c : fma(T.alpha, c, a.beta * *p);
                        }
                    } else {
                        sig[mb % SIG][nb][r] = fma(T.alpha, c, sig[mb % SIG][nb][r]);
                    }
                }
    }
    if (MODE == kModeAccum) {
#pragma unroll
        for (int mb = 0; mb < SIG; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = m0 + wm * 64 + mb * 16 + 4 * r + lq;
                    const int j = n0 + wn * 64 + nb * 16 + l16;
                    if (i < out.M && j < out.N)
                        out.C[static_cast<int64_t>(i) * out.ldc + j] = sig[mb][nb][r];
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

template <bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void k_dgemm_single(Dgemm64Args a, int tiles_m) {
    __shared__ double lds[4 * kBK * kLd];
    int tm, tn;
    tile_order(blockIdx.x, tiles_m, a.tiles_n, tm, tn);
    const Term64 term = a.term;
    dgemm_tile<TA, TB, kModeGemm>(a, [&](int) { return term; }, 0, 1, a.out, tm * kBM, tn * kBN, lds);
}

template <bool TB, int MODE>
__global__ __launch_bounds__(256, MODE == kModeAccum ? 1 : 2) void k_dgemm_grouped(Dgemm64Args a) {
    __shared__ double lds[4 * kBK * kLd];
    const TileDesc td = a.tiles[blockIdx.x];
    if (td.out < 0) return;  // padding of the XCD order
    OutDesc od = a.outs[td.out];
    if (a.out_base) od.C = a.out_base + reinterpret_cast<intptr_t>(od.C);
    const Term64 *terms = a.terms;
    const double *b_base = a.b_base;
    dgemm_tile<false, TB, MODE>(a,
                          [&](int i) {
                              Term64 tm = terms[i];
                              if (b_base) tm.B = b_base + reinterpret_cast<intptr_t>(tm.B);
                              return tm;
                          },
                          td.term_begin, td.term_end, od, td.m0, td.n0, lds);
}

}  // namespace

PairShape dgemm_shape() { return PairShape{kBM, kBN}; }

hipError_t launch_dgemm_single(bool ta, bool tb, const Dgemm64Args &a, int tiles_m,
                               hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(tiles_m) * static_cast<unsigned>(a.tiles_n);
    if (grid == 0) return hipSuccess;
    if (!ta && !tb) hipLaunchKernelGGL((k_dgemm_single<false, false>), dim3(grid), dim3(256), 0, s, a, tiles_m);
    if (!ta && tb) hipLaunchKernelGGL((k_dgemm_single<false, true>), dim3(grid), dim3(256), 0, s, a, tiles_m);
    if (ta && !tb) hipLaunchKernelGGL((k_dgemm_single<true, false>), dim3(grid), dim3(256), 0, s, a, tiles_m);
    if (ta && tb) hipLaunchKernelGGL((k_dgemm_single<true, true>), dim3(grid), dim3(256), 0, s, a, tiles_m);
    return hipGetLastError();
}

hipError_t launch_dgemm_grouped(bool tb, const Dgemm64Args &a, int grid, hipStream_t s) {
    (void)grid;
    if (a.ntiles == 0) return hipSuccess;
    const bool acc = a.mode == kModeAccum;
    if (tb && acc) hipLaunchKernelGGL((k_dgemm_grouped<true, kModeAccum>), dim3(a.ntiles), dim3(256), 0, s, a);
    if (tb && !acc) hipLaunchKernelGGL((k_dgemm_grouped<true, kModeGemm>), dim3(a.ntiles), dim3(256), 0, s, a);
    if (!tb && acc) hipLaunchKernelGGL((k_dgemm_grouped<false, kModeAccum>), dim3(a.ntiles), dim3(256), 0, s, a);
    if (!tb && !acc) hipLaunchKernelGGL((k_dgemm_grouped<false, kModeGemm>), dim3(a.ntiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace oz
