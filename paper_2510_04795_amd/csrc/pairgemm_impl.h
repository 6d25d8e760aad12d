// Steps 3 and 4 of the emulated GEMM ("Theory of emulated FP64 arithmetic"):
// every kept slice pair (s, t), s + t < G, multiplied exactly on the int8
// matrix cores with int32 accumulation, one accumulator set per diagonal
// g = s + t (all pairs of a diagonal carry the same weight 2^-8g), then the
// fused FP64 recombination per output element
//
//     h = Q_{G-1};  h = fma(h, 2^-8, Q_g) for g = G-2 .. 0   (the multiply is exact)
//     c = ldexp(h, e_i + f_j - 14)
//
// followed by the output rule of the mode (plain GEMM with alpha/beta, an
// ordered sum of terms for the effective Hamiltonian, raw Q for tests, or
// int64 carry of a K chunk).
//
// Tiling.  256 threads = 2 x 2 waves, one wave per SIMD; a wave owns MB x NB
// blocks of 32 x 32 outputs (v_mfma_i32_32x32x32_i8) for all G diagonals, so
// the block tile is (64 MB) x (64 NB).  The inner dimension advances one
// packed 32-wide K block at a time through a double-buffered LDS stage that
// is filled by direct global->LDS 16-byte loads (no staging registers): the
// loads of block kb + 1 are in flight while block kb is multiplied, with one
// barrier per block.  A stage is the 2S runs of A rows and of B rows exactly
// as they are stored (internal.h), so every MFMA operand is one 1 KiB read of
// consecutive LDS addresses.  Rows past the operand are clamped to its last
// padded row: they only feed outputs that are never stored.
#pragma once

#include "internal.h"

namespace oz {
namespace pair {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;

template <int S, int G, int MB, int NB>
struct Cfg {
    static constexpr int BM = 2 * MB * 32;
    static constexpr int BN = 2 * NB * 32;
    static constexpr int STAGE = 2 * S * (BM + BN);     // uint4 per LDS stage
    static constexpr int A_SEG = 2 * S * BM / 64;       // 64-row wave loads for A
    static constexpr int SEGS = 2 * S * (BM + BN) / 64; // all wave loads per stage
};

// Direct-to-LDS loads of one packed K block: the stage holds 2S runs of BM
// A rows then 2S runs of BN B rows; every wave issues 64-row segments (one
// 16-byte chunk per lane).  The per-wave segment list is fixed for a term, so
// it is computed once: a lane address at block 0, the per-block stride and
// the LDS offset of each segment the wave owns.
template <int S, int G, int MB, int NB>
struct LoadPlan {
    using C = Cfg<S, G, MB, NB>;
    static constexpr int NL = (C::SEGS + 3) / 4;
    const uint4 *src[NL];
    int64_t stride[NL];
    int lds_off[NL];
    bool valid[NL];

    __device__ __forceinline__ void init(const uint4 *gA, const uint4 *gB, int64_t a_rows_p,
                                         int64_t b_rows_p, int m0, int n0, int wave, int lane) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int q = wave + 4 * i;
            valid[i] = q < C::SEGS;
            if (q < C::A_SEG) {
                const int run = q / (C::BM / 64);
                const int seg = q - run * (C::BM / 64);
                int64_t row = m0 + seg * 64 + lane;
                row = row < a_rows_p ? row : a_rows_p - 1;
                src[i] = gA + run * a_rows_p + row;
                stride[i] = 2 * S * a_rows_p;
                lds_off[i] = run * C::BM + seg * 64;
            } else {
                const int qb = (q < C::SEGS ? q : C::A_SEG) - C::A_SEG;
                const int run = qb / (C::BN / 64);
                const int seg = qb - run * (C::BN / 64);
                int64_t row = n0 + seg * 64 + lane;
                row = row < b_rows_p ? row : b_rows_p - 1;
                src[i] = gB + run * b_rows_p + row;
                stride[i] = 2 * S * b_rows_p;
                lds_off[i] = 2 * S * C::BM + run * C::BN + seg * 64;
            }
        }
    }

    __device__ __forceinline__ void issue(uint4 *stage, int kb) const {
#pragma unroll
        for (int i = 0; i < NL; ++i)
            if (valid[i])
                __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src[i] + kb * stride[i]),
                                                 (lds_void *)(stage + lds_off[i]), 16, 0, 0);
    }
};

// All kept pair products of one LDS stage (one 32-wide K block).  The B
// fragments of every kept slice stay in registers; A fragments are streamed
// one slice at a time, so operands cost 4 S NB + 4 MB registers.
template <int S, int G, int MB, int NB>
__device__ __forceinline__ void multiply_stage(v16i (&acc)[G][MB][NB], const uint4 *stage, int wm,
                                               int wn, int half, int l32) {
    using C = Cfg<S, G, MB, NB>;
    constexpr int TB = S < G ? S : G;  // B slices that meet at least one kept pair
    const uint4 *sA = stage;
    const uint4 *sB = stage + 2 * S * C::BM;
    v4i bf[TB][NB];
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const uint4 v = sB[(t * 2 + half) * C::BN + (wn * NB + nb) * 32 + l32];
            bf[t][nb] = v4i{static_cast<int>(v.x), static_cast<int>(v.y), static_cast<int>(v.z),
                            static_cast<int>(v.w)};
        }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (s >= G) continue;
        v4i af[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const uint4 v = sA[(s * 2 + half) * C::BM + (wm * MB + mb) * 32 + l32];
            af[mb] = v4i{static_cast<int>(v.x), static_cast<int>(v.y), static_cast<int>(v.z),
                         static_cast<int>(v.w)};
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            if (s + t >= G) continue;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[s + t][mb][nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                        af[mb], bf[t][nb], acc[s + t][mb][nb], 0, 0, 0);
        }
    }
}

// Exact diagonal sums of one tile for one term, accumulated over all K blocks.
template <int S, int G, int MB, int NB>
__device__ __forceinline__ void pair_mainloop(v16i (&acc)[G][MB][NB], uint4 *lds0, uint4 *lds1,
                                              const TermDesc &T, int m0, int n0) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
    const int wm = wave >> 1;
    const int wn = wave & 1;
    const int half = lane >> 5;
    const int l32 = lane & 31;
    const uint4 *gA = reinterpret_cast<const uint4 *>(T.A);
    const uint4 *gB = reinterpret_cast<const uint4 *>(T.B);
    const int nkb = T.kblocks;

#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[g][mb][nb] = v16i{};
    if (nkb == 0) return;

    LoadPlan<S, G, MB, NB> lp;
    lp.init(gA, gB, T.a_rows_p, T.b_rows_p, m0, n0, wave, lane);
    lp.issue(lds0, 0);
    // Blocks are taken two at a time (stage 0, stage 1) so each LDS stage is
    // its own object; the loop has a single exit and an odd last block is
    // peeled, which keeps the accumulators in place across iterations.
    int kb = 0;
    for (; kb + 2 <= nkb; kb += 2) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        lp.issue(lds1, kb + 1);
        multiply_stage<S, G, MB, NB>(acc, lds0, wm, wn, half, l32);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (kb + 2 < nkb) lp.issue(lds0, kb + 2);
        multiply_stage<S, G, MB, NB>(acc, lds1, wm, wn, half, l32);
    }
    if (kb < nkb) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        multiply_stage<S, G, MB, NB>(acc, lds0, wm, wn, half, l32);
    }
}

// FP64 value of one output element from its diagonal sums (plus int64 carries).
template <int G>
__device__ __forceinline__ double horner(const long long (&q)[G], int32_t ei, int32_t fj) {
    if (ei == kExpBad || fj == kExpBad) return __longlong_as_double(0x7ff8000000000000ll);
    double h = static_cast<double>(q[G - 1]);
#pragma unroll
    for (int g = G - 2; g >= 0; --g) h = fma(h, 0x1p-8, static_cast<double>(q[g]));
    return ldexp(h, ei + fj - 14);
}

template <int S, int G, int MB, int NB, int MODE, typename GetTerm>
__device__ __forceinline__ void pair_tile(const PairArgs &a, GetTerm get_term, int tb, int te,
                                          const OutDesc &out, int m0, int n0, uint4 *lds0,
                                          uint4 *lds1) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave >> 1;
    const int wn = wave & 1;
    const int half = lane >> 5;
    const int l32 = lane & 31;

    constexpr int SIG = (MODE == kModeAccum) ? 16 : 1;
    double sig[MB][NB][SIG];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int r = 0; r < SIG; ++r) sig[mb][nb][r] = 0.0;

    // only the accumulating mode sums several terms into one tile
    const int tend = (MODE == kModeAccum) ? te : tb + 1;
    for (int ti = tb; ti < tend; ++ti) {
        const TermDesc T = get_term(ti);
        v16i acc[G][MB][NB];
        pair_mainloop<S, G, MB, NB>(acc, lds0, lds1, T, m0, n0);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int j = n0 + (wn * NB + nb) * 32 + l32;
            const bool jok = j < out.N;
            int32_t fj = 0;
            if (MODE != kModeQ && MODE != kModeQ64 && jok) fj = T.f[j];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    // keep one element's recombination at a time in registers
                    __builtin_amdgcn_sched_barrier(0);
                    const int i = m0 + (wm * MB + mb) * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                    const bool ok = jok && i < out.M;
                    if (MODE == kModeQ) {
                        if (ok) {
                            const int64_t plane = static_cast<int64_t>(out.M) * out.N;
#pragma unroll
                            for (int g = 0; g < G; ++g)
                                a.Q[g * plane + static_cast<int64_t>(i) * out.N + j] = acc[g][mb][nb][r];
                        }
                    } else if (MODE == kModeQ64) {
                        const int64_t idx = static_cast<int64_t>(i) * a.qw_ld + j;
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            int64_t *p = a.Qw + g * a.qw_plane + idx;
                            const long long v = acc[g][mb][nb][r];
                            *p = a.qw_first ? v : *p + v;
                        }
                    } else {
                        if (!ok) continue;
                        long long q[G];
#pragma unroll
                        for (int g = 0; g < G; ++g) q[g] = acc[g][mb][nb][r];
                        if (MODE == kModeGemm && a.Qw) {
                            const int64_t idx = static_cast<int64_t>(i) * a.qw_ld + j;
#pragma unroll
                            for (int g = 0; g < G; ++g) q[g] += a.Qw[g * a.qw_plane + idx];
                        }
                        const double c = horner<G>(q, T.e[i], fj);
                        if (MODE == kModeGemm) {
                            double *p = out.C + static_cast<int64_t>(i) * out.ldc + j;
                            *p = (a.beta == 0.0) ? T.alpha * c : fma(T.alpha, c, a.beta * *p);
                        } else {
                            sig[mb][nb][r % SIG] = fma(T.alpha, c, sig[mb][nb][r % SIG]);
                        }
                    }
                }
        }
    }

    if (MODE == kModeAccum) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < SIG; ++r) {
                    const int i = m0 + (wm * MB + mb) * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                    const int j = n0 + (wn * NB + nb) * 32 + l32;
                    if (i < out.M && j < out.N)
                        out.C[static_cast<int64_t>(i) * out.ldc + j] = sig[mb][nb][r];
                }
    }
}

// Tile index -> (tm, tn).  Blocks are dispatched to the 8 XCDs round robin;
// give every XCD a contiguous range of tiles, walked in groups of 8 tile rows,
// so the blocks sharing an L2 also share A and B panels.
__device__ __forceinline__ void tile_coords(int b, int tiles_m, int tiles_n, int &tm, int &tn) {
    const int T = tiles_m * tiles_n;
    const int nx = 8;
    const int q = T / nx;
    const int rem = T - q * nx;
    const int x = b % nx;
    const int idx = b / nx;
    const int lin = x * q + (x < rem ? x : rem) + idx;
    const int group = 8;
    const int per_group = group * tiles_n;
    const int gid = lin / per_group;
    const int first = gid * group;
    const int rows = tiles_m - first < group ? tiles_m - first : group;
    const int w = lin - gid * per_group;
    tm = first + w % rows;
    tn = w / rows;
}

template <int S, int G, int MB, int NB, int MODE>
__global__ __launch_bounds__(256) void k_pair_single(PairArgs a, int tiles_m) {
    using C = Cfg<S, G, MB, NB>;
    __shared__ uint4 lds0[C::STAGE];
    __shared__ uint4 lds1[C::STAGE];
    int tm, tn;
    tile_coords(blockIdx.x, tiles_m, a.tiles_n, tm, tn);
    const TermDesc term = a.term;
    pair_tile<S, G, MB, NB, MODE>(a, [&](int) { return term; }, 0, 1, a.out, tm * C::BM,
                                  tn * C::BN, lds0, lds1);
}

// One block per listed tile (tiles are listed longest first).
template <int S, int G, int MB, int NB, int MODE>
__global__ __launch_bounds__(256) void k_pair_grouped(PairArgs a) {
    using C = Cfg<S, G, MB, NB>;
    __shared__ uint4 lds0[C::STAGE];
    __shared__ uint4 lds1[C::STAGE];
    const TileDesc td = a.tiles[blockIdx.x];
    OutDesc od = a.outs[td.out];
    if (a.out_base) od.C = a.out_base + reinterpret_cast<intptr_t>(od.C);
    const TermDesc *terms = a.terms;
    pair_tile<S, G, MB, NB, MODE>(a, [&](int i) { return terms[i]; }, td.term_begin, td.term_end,
                                  od, td.m0, td.n0, lds0, lds1);
}

// Per-(S, G) tile shape: as wide as the accumulators allow.
// Wave-tile variants (MB x NB blocks of 32 x 32 per wave).  The 1 x 1
// variant is always built; a wider one only when its G accumulator sets fit
// in 192 registers (16 G MB NB), leaving the rest of the register file to
// operands and addresses.
constexpr int kNumVariants = 4;
__host__ __device__ constexpr int variant_mb(int v) { return v == 1 || v == 3 ? 2 : 1; }
__host__ __device__ constexpr int variant_nb(int v) { return v == 2 || v == 3 ? 2 : 1; }
__host__ __device__ constexpr bool variant_fits(int G, int v) {
    return v == 0 || 16 * G * variant_mb(v) * variant_nb(v) <= 192;
}
// default: the widest tile that fits, preferring 2 x 1
__host__ __device__ constexpr int default_variant(int G) {
    return variant_fits(G, 3) ? 3 : (variant_fits(G, 1) ? 1 : 0);
}

template <int S, int G, int V>
hipError_t run_single_v(const PairArgs &a, int tiles_m, hipStream_t s) {
    constexpr int MB = variant_mb(V), NB = variant_nb(V);
    if constexpr (!variant_fits(G, V)) {
        return hipErrorInvalidValue;
    } else {
        const unsigned grid = static_cast<unsigned>(tiles_m) * static_cast<unsigned>(a.tiles_n);
        if (grid == 0) return hipSuccess;
        switch (a.mode) {
            case kModeGemm:
                hipLaunchKernelGGL((k_pair_single<S, G, MB, NB, kModeGemm>), dim3(grid), dim3(256), 0, s, a, tiles_m);
                break;
            case kModeQ:
                hipLaunchKernelGGL((k_pair_single<S, G, MB, NB, kModeQ>), dim3(grid), dim3(256), 0, s, a, tiles_m);
                break;
            case kModeQ64:
                hipLaunchKernelGGL((k_pair_single<S, G, MB, NB, kModeQ64>), dim3(grid), dim3(256), 0, s, a, tiles_m);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}

template <int S, int G, int V>
hipError_t run_grouped_v(const PairArgs &a, hipStream_t s) {
    constexpr int MB = variant_mb(V), NB = variant_nb(V);
    if constexpr (!variant_fits(G, V)) {
        return hipErrorInvalidValue;
    } else {
        if (a.ntiles == 0) return hipSuccess;
        switch (a.mode) {
            case kModeGemm:
                hipLaunchKernelGGL((k_pair_grouped<S, G, MB, NB, kModeGemm>), dim3(a.ntiles), dim3(256), 0, s, a);
                break;
            case kModeAccum:
                hipLaunchKernelGGL((k_pair_grouped<S, G, MB, NB, kModeAccum>), dim3(a.ntiles), dim3(256), 0, s, a);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}

template <int S, int G>
hipError_t run_single(int v, const PairArgs &a, int tiles_m, hipStream_t s) {
    switch (v) {
        case 0: return run_single_v<S, G, 0>(a, tiles_m, s);
        case 1: return run_single_v<S, G, 1>(a, tiles_m, s);
        case 2: return run_single_v<S, G, 2>(a, tiles_m, s);
        case 3: return run_single_v<S, G, 3>(a, tiles_m, s);
        default: return hipErrorInvalidValue;
    }
}

template <int S, int G>
hipError_t run_grouped(int v, const PairArgs &a, hipStream_t s) {
    switch (v) {
        case 0: return run_grouped_v<S, G, 0>(a, s);
        case 1: return run_grouped_v<S, G, 1>(a, s);
        case 2: return run_grouped_v<S, G, 2>(a, s);
        case 3: return run_grouped_v<S, G, 3>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pair

// Per-S entry points (pairgemm_s<S>.hip).
#define OZ_DECLARE_PAIR_S(S_)                                                                   \
    hipError_t pair_single_s##S_(int G, int v, const PairArgs &a, int tiles_m, hipStream_t s);  \
    hipError_t pair_grouped_s##S_(int G, int v, const PairArgs &a, hipStream_t s);
OZ_DECLARE_PAIR_S(2)
OZ_DECLARE_PAIR_S(3)
OZ_DECLARE_PAIR_S(4)
OZ_DECLARE_PAIR_S(5)
OZ_DECLARE_PAIR_S(6)
OZ_DECLARE_PAIR_S(7)
OZ_DECLARE_PAIR_S(8)
#undef OZ_DECLARE_PAIR_S

// Instantiate the three diagonal counts G = S, S + 1, 2S - 1 for one S.
#define OZ_DEFINE_PAIR_S(S_)                                                                    \
    hipError_t pair_single_s##S_(int G, int v, const PairArgs &a, int tiles_m, hipStream_t s) { \
        if (G == S_) return pair::run_single<S_, S_>(v, a, tiles_m, s);                         \
        if (G == S_ + 1) return pair::run_single<S_, S_ + 1>(v, a, tiles_m, s);                 \
        if (G == 2 * S_ - 1) return pair::run_single<S_, 2 * S_ - 1>(v, a, tiles_m, s);         \
        return hipErrorInvalidValue;                                                            \
    }                                                                                           \
    hipError_t pair_grouped_s##S_(int G, int v, const PairArgs &a, hipStream_t s) {             \
        if (G == S_) return pair::run_grouped<S_, S_>(v, a, s);                                 \
        if (G == S_ + 1) return pair::run_grouped<S_, S_ + 1>(v, a, s);                         \
        if (G == 2 * S_ - 1) return pair::run_grouped<S_, 2 * S_ - 1>(v, a, s);                 \
        return hipErrorInvalidValue;                                                            \
    }

}  // namespace oz
