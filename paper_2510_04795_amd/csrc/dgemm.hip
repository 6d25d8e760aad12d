// Native FP64 GEMM on the FP64 matrix cores (v_mfma_f64_16x16x4_f64): the
// comparator for the emulated path and the slices = 0 mode of every entry
// point.  Any summation order is a valid FP64 GEMM, so this path is checked
// against the textbook gamma_K |A||B| bound, not bit for bit.
//
// Operand layout of the 16x16x4 instruction (measured): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register r of lane l
// holds C[4 r + l / 16][l % 16].
//
// Tile: 256 threads = 2 x 2 waves, 64 x 64 outputs, each wave 2 x 2 blocks of
// 16 x 16; K staged through LDS 16 at a time (k-major, so both operand reads
// are 16 consecutive doubles per quarter wave).
#include "internal.h"

namespace oz {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kBM = 64;
constexpr int kBN = 64;
constexpr int kBK = 16;
constexpr int kPad = 4;

template <bool TA, bool TB, typename GetTerm>
__device__ __forceinline__ void dgemm_tile(const Dgemm64Args &a, GetTerm get_term, int tb, int te,
                                           const OutDesc &out, int m0, int n0,
                                           double (*sA)[kBM + kPad], double (*sB)[kBN + kPad]) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1;
    const int wn = wave & 1;
    const int lq = lane >> 4;   // 0..3
    const int l16 = lane & 15;

    double sig[2][2][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) sig[mb][nb][r] = 0.0;

    for (int ti = tb; ti < te; ++ti) {
        const Term64 T = get_term(ti);
        v4d acc[2][2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = v4d{0.0, 0.0, 0.0, 0.0};
        const int K = T.K;
        for (int k0 = 0; k0 < K; k0 += kBK) {
            __syncthreads();
            if (!TA) {
                const int i = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int gi = m0 + i, gk = k0 + kk + x;
                    sA[kk + x][i] = (gi < out.M && gk < K) ? T.A[static_cast<int64_t>(gi) * T.lda + gk] : 0.0;
                }
            } else {
                const int k = tid >> 4, ii = (tid & 15) * 4;
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int gi = m0 + ii + x, gk = k0 + k;
                    sA[k][ii + x] = (gi < out.M && gk < K) ? T.A[static_cast<int64_t>(gk) * T.lda + gi] : 0.0;
                }
            }
            if (!TB) {
                const int k = tid >> 4, jj = (tid & 15) * 4;
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int gj = n0 + jj + x, gk = k0 + k;
                    sB[k][jj + x] = (gj < out.N && gk < K) ? T.B[static_cast<int64_t>(gk) * T.ldb + gj] : 0.0;
                }
            } else {
                const int j = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int gj = n0 + j, gk = k0 + kk + x;
                    sB[kk + x][j] = (gj < out.N && gk < K) ? T.B[static_cast<int64_t>(gj) * T.ldb + gk] : 0.0;
                }
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < kBK / 4; ++ks) {
                double af[2], bf[2];
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) af[mb] = sA[ks * 4 + lq][wm * 32 + mb * 16 + l16];
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) bf[nb] = sB[ks * 4 + lq][wn * 32 + nb * 16 + l16];
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb)
                        acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mb], bf[nb],
                                                                           acc[mb][nb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = m0 + wm * 32 + mb * 16 + 4 * r + lq;
                    const int j = n0 + wn * 32 + nb * 16 + l16;
                    const double c = acc[mb][nb][r];
                    if (a.mode == kModeGemm) {
                        if (i < out.M && j < out.N) {
                            double *p = out.C + static_cast<int64_t>(i) * out.ldc + j;
                            *p = (a.beta == 0.0) ? T.alpha * c : fma(T.alpha, c, a.beta * *p);
                        }
                    } else {
                        sig[mb][nb][r] = fma(T.alpha, c, sig[mb][nb][r]);
                    }
                }
    }
    if (a.mode == kModeAccum) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = m0 + wm * 32 + mb * 16 + 4 * r + lq;
                    const int j = n0 + wn * 32 + nb * 16 + l16;
                    if (i < out.M && j < out.N)
                        out.C[static_cast<int64_t>(i) * out.ldc + j] = sig[mb][nb][r];
                }
    }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_dgemm_single(Dgemm64Args a) {
    __shared__ double sA[kBK][kBM + kPad];
    __shared__ double sB[kBK][kBN + kPad];
    const int tm = blockIdx.x / a.tiles_n;
    const int tn = blockIdx.x - tm * a.tiles_n;
    const Term64 term = a.term;
    dgemm_tile<TA, TB>(a, [&](int) { return term; }, 0, 1, a.out, tm * kBM, tn * kBN, sA, sB);
}

template <bool TB>
__global__ __launch_bounds__(256) void k_dgemm_grouped(Dgemm64Args a) {
    __shared__ double sA[kBK][kBM + kPad];
    __shared__ double sB[kBK][kBN + kPad];
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const TileDesc td = a.tiles[t];
        if (td.out < 0) continue;  // padding of the XCD order
        OutDesc od = a.outs[td.out];
        if (a.out_base) od.C = a.out_base + reinterpret_cast<intptr_t>(od.C);
        const Term64 *terms = a.terms;
        const double *b_base = a.b_base;
        dgemm_tile<false, TB>(a,
                              [&](int i) {
                                  Term64 tm = terms[i];
                                  if (b_base) tm.B = b_base + reinterpret_cast<intptr_t>(tm.B);
                                  return tm;
                              },
                              td.term_begin, td.term_end, od, td.m0, td.n0, sA, sB);
        __syncthreads();
    }
}

}  // namespace

PairShape dgemm_shape() { return PairShape{kBM, kBN}; }

hipError_t launch_dgemm_single(bool ta, bool tb, const Dgemm64Args &a, int tiles_m,
                               hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(tiles_m) * static_cast<unsigned>(a.tiles_n);
    if (grid == 0) return hipSuccess;
    if (!ta && !tb) hipLaunchKernelGGL((k_dgemm_single<false, false>), dim3(grid), dim3(256), 0, s, a);
    if (!ta && tb) hipLaunchKernelGGL((k_dgemm_single<false, true>), dim3(grid), dim3(256), 0, s, a);
    if (ta && !tb) hipLaunchKernelGGL((k_dgemm_single<true, false>), dim3(grid), dim3(256), 0, s, a);
    if (ta && tb) hipLaunchKernelGGL((k_dgemm_single<true, true>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dgemm_grouped(bool tb, const Dgemm64Args &a, int grid, hipStream_t s) {
    if (grid == 0 || a.ntiles == 0) return hipSuccess;
    if (tb)
        hipLaunchKernelGGL((k_dgemm_grouped<true>), dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_dgemm_grouped<false>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace oz
