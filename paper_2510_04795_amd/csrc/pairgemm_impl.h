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
// Tiling.  WM x WN waves (4, 8 or 16) per workgroup; a wave owns MB x NB
// blocks of 32 x 32 outputs (v_mfma_i32_32x32x32_i8) for all G diagonals, so
// the block tile is (32 WM MB) x (32 WN NB); the seven built shapes are
// listed with variant_fits below.  The inner dimension advances one packed
// 32-wide K block at a time through LDS stages filled by direct
// global->LDS 16-byte loads (no staging registers).  A stage is the 2S runs
// of A rows and of B rows exactly as they are stored (internal.h), so every
// MFMA operand is one 1 KiB read of consecutive LDS addresses.  Rows past
// the operand are clamped to its last padded row: they only feed outputs
// that are never stored.
//
// Main loops, chosen per shape at compile time from the register budget:
// the ring (one block per wave: three stages, loads two blocks ahead, or
// two stages and one block ahead where a third would cost the second
// workgroup per CU; explicit vmcnt waits, a bare s_barrier and one
// generated asm block per step from asm_steps.h), and two double-buffered
// loops for waves with several blocks (next block's fragments prefetched
// when two fragment sets fit, else read after the barrier).  The grouped,
// streamed, resident and paired-term kernels below run the same steps over
// tile and term lists.
#pragma once

#include <algorithm>

#include "internal.h"

namespace oz {
namespace pair {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;

}  // namespace pair
}  // namespace oz

#include "asm_steps.h"

namespace oz {
namespace pair {

// WM x WN waves per block, each owning MB x NB blocks of 32 x 32 outputs.
template <int S, int G, int WM, int WN, int MB, int NB>
struct Cfg {
    static constexpr int NW = WM * WN;                  // waves per block
    static constexpr int NT = 64 * NW;                  // threads per block
    static constexpr int BM = WM * MB * 32;
    static constexpr int BN = WN * NB * 32;
    static constexpr int STAGE = 2 * S * (BM + BN);     // uint4 per LDS stage
    static constexpr int A_SEG = 2 * S * BM / 64;       // 64-row wave loads for A
    static constexpr int SEGS = 2 * S * (BM + BN) / 64; // all wave loads per stage
    static constexpr int STAGE_BYTES = STAGE * 16;
    // loads every wave issues per stage (some waves issue one more)
    static constexpr int NL_MIN = SEGS / NW;
    // s_waitcnt immediates: vmcnt(n) (bits 3:0 and 15:14) with lgkmcnt(0)
    // (bits 11:8) and expcnt at its maximum (bits 6:4)
    static constexpr int wait_vm(int n) { return (n & 15) | (((n >> 4) & 3) << 14) | (7 << 4); }
    static constexpr int WAIT_ALL = wait_vm(0);
    static constexpr int WAIT_NEWEST = wait_vm(NL_MIN);      // one block's loads may stay in flight
    static constexpr int WAIT_NEWER2 = wait_vm(2 * NL_MIN);  // two blocks' loads may stay in flight
    static constexpr int WAIT_LDS = wait_vm(63);              // lgkmcnt(0) only
};

// Direct-to-LDS loads of one packed K block: the stage holds 2S runs of BM
// A rows then 2S runs of BN B rows; every wave issues 64-row segments (one
// 16-byte chunk per lane).  The loads are buffer loads with an LDS
// destination: one buffer descriptor per operand and K block (scalar), and
// per segment a fixed lane offset within the K block, so the per-lane
// registers stay the same for the whole loop.
constexpr int kBufferDword3 = 0x00020000;  // raw buffer, 32-bit data format

// Tag only separates specializations: the streamed kernel uses its own
// (Tag = 1).  With one shared specialization, hipcc's host pass silently
// dropped the streamed kernel's host stub (the library then failed to load
// with an undefined symbol).
template <int S, int G, int WM, int WN, int MB, int NB, int Tag = 0>
struct LoadPlan {
    using C = Cfg<S, G, WM, WN, MB, NB>;
    static constexpr int NL = (C::SEGS + C::NW - 1) / C::NW;
    const char *A, *B;
    int a_kb_bytes, b_kb_bytes;  // bytes of one packed K block of each operand
    int voff[NL];                // lane byte offset within the K block
    int lds_off[NL];             // uint4 offset of the segment in a stage
    bool valid[NL], isA[NL];     // uniform per wave

    __device__ __forceinline__ void init(const void *gA, const void *gB, int64_t a_rows_p,
                                         int64_t b_rows_p, int m0, int n0, int wave, int lane) {
        A = static_cast<const char *>(gA);
        B = static_cast<const char *>(gB);
        a_kb_bytes = static_cast<int>(2 * S * a_rows_p * 16);
        b_kb_bytes = static_cast<int>(2 * S * b_rows_p * 16);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int q = wave + C::NW * i;
            valid[i] = q < C::SEGS;
            isA[i] = q < C::A_SEG;
            if (q < C::A_SEG) {
                const int run = q / (C::BM / 64);
                const int seg = q - run * (C::BM / 64);
                int64_t row = m0 + seg * 64 + lane;
                row = row < a_rows_p ? row : a_rows_p - 1;
                voff[i] = static_cast<int>((run * a_rows_p + row) * 16);
                lds_off[i] = run * C::BM + seg * 64;
            } else {
                const int qb = (q < C::SEGS ? q : C::A_SEG) - C::A_SEG;
                const int run = qb / (C::BN / 64);
                const int seg = qb - run * (C::BN / 64);
                int64_t row = n0 + seg * 64 + lane;
                row = row < b_rows_p ? row : b_rows_p - 1;
                voff[i] = static_cast<int>((run * b_rows_p + row) * 16);
                lds_off[i] = 2 * S * C::BM + run * C::BN + seg * 64;
            }
        }
    }

    __device__ __forceinline__ void issue(uint4 *stage, int kb) const {
        const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char *>(A + static_cast<int64_t>(kb) * a_kb_bytes), 0, a_kb_bytes, kBufferDword3);
        const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char *>(B + static_cast<int64_t>(kb) * b_kb_bytes), 0, b_kb_bytes, kBufferDword3);
#pragma unroll
        for (int i = 0; i < NL; ++i)
            if (valid[i])
                __builtin_amdgcn_raw_ptr_buffer_load_lds(isA[i] ? ra : rb, (lds_void *)(stage + lds_off[i]), 16,
                                                         voff[i], 0, 0, 0);
    }
};

typedef __attribute__((address_space(4))) const TermDesc ConstTermDesc;

// Term i of a list that does not change during the launch, read through the
// constant address space so the reads go to scalar registers (a vector load
// would have to wait for every load into LDS issued before it).
__device__ __forceinline__ TermDesc const_term(const TermDesc *list, int i) {
    const ConstTermDesc *c = (const ConstTermDesc *)reinterpret_cast<uintptr_t>(list + i);
    TermDesc t;
    t.A = c->A;
    t.e = c->e;
    t.B = c->B;
    t.f = c->f;
    t.a_rows_p = c->a_rows_p;
    t.b_rows_p = c->b_rows_p;
    t.kblocks = c->kblocks;
    t.pad_ = 0;
    t.alpha = c->alpha;
    return t;
}

// Operand fragments of one stage for one wave: every slice that meets a
// kept pair, for the wave's MB row blocks (A) and NB column blocks (B).
// Each fragment is one 16-byte LDS read per lane (a 1 KiB run).
template <int S, int G, int MB, int NB>
struct Frags {
    static constexpr int T = S < G ? S : G;  // slices that meet at least one kept pair
    v4i a[T][MB];
    v4i b[T][NB];
};

__device__ __forceinline__ v4i lds_frag(const uint4 *p) {
    const uint4 v = *p;
    return v4i{static_cast<int>(v.x), static_cast<int>(v.y), static_cast<int>(v.z), static_cast<int>(v.w)};
}

// All fragments of one stage, in the order the MFMAs consume them (A slice
// 0 and every B slice, then A slices 1, 2, ...), so each MFMA waits only for
// its own operands.
template <int S, int G, int WM, int WN, int MB, int NB, typename F>
__device__ __forceinline__ void read_stage(F &f, const uint4 *stage, int wm, int wn, int half, int l32) {
    using C = Cfg<S, G, WM, WN, MB, NB>;
    const uint4 *sA = stage;
    const uint4 *sB = stage + 2 * S * C::BM;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) f.a[0][mb] = lds_frag(sA + half * C::BM + (wm * MB + mb) * 32 + l32);
#pragma unroll
    for (int t = 0; t < F::T; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            f.b[t][nb] = lds_frag(sB + (t * 2 + half) * C::BN + (wn * NB + nb) * 32 + l32);
#pragma unroll
    for (int s = 1; s < F::T; ++s)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            f.a[s][mb] = lds_frag(sA + (s * 2 + half) * C::BM + (wm * MB + mb) * 32 + l32);
}

// Number of kept pairs (s, t), s + t < G, both below min(S, G).
template <int S, int G>
constexpr int kept_pairs() {
    int n = 0;
    for (int s = 0; s < S && s < G; ++s)
        for (int t = 0; t < S && t < G; ++t)
            if (s + t < G) ++n;
    return n;
}

// Pairs of a stage deferred to the next one: they run while the next
// stage's fragments are on their way from LDS.  A 2 x 2 block of pairs
// ((0,0), (0,1), (1,0), (1,1)) needs only four fragments kept across the
// stage boundary.
template <int S, int G>
__host__ __device__ constexpr bool deferred_pair(int s, int t) {
    return kept_pairs<S, G>() >= 8 ? (s < 2 && t < 2) : (s == 0 && t == 0);
}

// The MFMAs of the kept pairs that are (DEFERRED) or are not (!DEFERRED)
// deferred, slice-major ((0,0), (0,1), ..., (1,0), ...): consecutive MFMAs
// feed different diagonals, and slice s of A is needed only once slice
// s - 1 is done.
template <bool DEFERRED, int S, int G, int MB, int NB, typename F>
__device__ __forceinline__ void mfma_pairs(v16i (&acc)[G][MB][NB], const F &f) {
#pragma unroll
    for (int s = 0; s < F::T; ++s)
#pragma unroll
        for (int t = 0; t < F::T; ++t) {
            if (s + t >= G || deferred_pair<S, G>(s, t) != DEFERRED) continue;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[s + t][mb][nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[s][mb], f.b[t][nb],
                                                                               acc[s + t][mb][nb], 0, 0, 0);
        }
}

// One K block in LDS stage `cur`.  After the barrier (block kb complete in
// `cur`, every wave done with `nxt`), all of its fragments are read, then
// the loads of block kb + 1 into `nxt` are started, so no LDS read of this
// wave is ever issued while a load into LDS is pending.  The deferred pairs
// of block kb - 1 (fragments in f) run first, then this block's other
// pairs; f then holds this block's fragments.
template <int S, int G, int WM, int WN, int MB, int NB, typename F, typename LP>
__device__ __forceinline__ void stage_step(v16i (&acc)[G][MB][NB], F &f, const uint4 *cur, uint4 *nxt,
                                           const LP &lp, int kb, int nkb, int wm, int wn, int half,
                                           int l32) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    F g;
    read_stage<S, G, WM, WN, MB, NB>(g, cur, wm, wn, half, l32);
    if (kb + 1 < nkb) lp.issue(nxt, kb + 1);
    __builtin_amdgcn_sched_barrier(0);
    mfma_pairs<true, S, G, MB, NB>(acc, f);
    mfma_pairs<false, S, G, MB, NB>(acc, g);
    __builtin_amdgcn_sched_barrier(0);
    f = g;
}

// One K block of the prefetching main loop.  On entry the fragments of block
// kb are in `cur` (their reads may still be in flight) and the loads of
// block kb + 1 into `rd` are in flight.  After the wait and the barrier
// (block kb + 1 complete in `rd`, every wave's reads of `fill` done), the
// fragments of block kb + 1 are read into `nxt`, the loads of block kb + 2
// into `fill` are started (after the reads in program order, so no LDS read
// is ever issued while a load into LDS is pending), and the MFMAs of block
// kb run from registers: the matrix cores start right after the barrier,
// and the LDS reads have the whole step to arrive.  The last step of a term
// also reads a set of fragments (nothing is pending on `rd` then; the
// values go unused), so every step is the same code and the accumulators
// keep their registers.
template <int S, int G, int WM, int WN, int MB, int NB, typename F, typename LP>
__device__ __forceinline__ void prefetch_step(v16i (&acc)[G][MB][NB], F &cur, uint4 *fill, const uint4 *rd,
                                           const LP &lp, int kb, int nkb, int wm, int wn, int half, int l32) {
    if (kb + 1 < nkb) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    F nxt;
    read_stage<S, G, WM, WN, MB, NB>(nxt, rd, wm, wn, half, l32);
    if (kb + 2 < nkb) lp.issue(fill, kb + 2);
    __builtin_amdgcn_sched_barrier(0);
    mfma_pairs<true, S, G, MB, NB>(acc, cur);
    mfma_pairs<false, S, G, MB, NB>(acc, cur);
    __builtin_amdgcn_sched_barrier(0);
    cur = nxt;
}

// Exact diagonal sums of one tile for one term, with the fragments read at
// the start of each block (stage_step).
template <int S, int G, int WM, int WN, int MB, int NB>
__device__ __forceinline__ void pair_mainloop_direct(v16i (&acc)[G][MB][NB], uint4 *lds0, uint4 *lds1,
                                              const TermDesc &T, int m0, int n0) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
    const int wm = wave / WN;
    const int wn = wave % WN;
    const int half = lane >> 5;
    const int l32 = lane & 31;
    const int nkb = T.kblocks;

#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[g][mb][nb] = v16i{};
    if (nkb == 0) return;

    LoadPlan<S, G, WM, WN, MB, NB> lp;
    lp.init(T.A, T.B, T.a_rows_p, T.b_rows_p, m0, n0, wave, lane);
    // a previous term of this block (accumulating mode) may still read the stages
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    lp.issue(lds0, 0);
    // no block before the first: its deferred pairs multiply zeros
    Frags<S, G, MB, NB> f;
#pragma unroll
    for (int s = 0; s < Frags<S, G, MB, NB>::T; ++s) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) f.a[s][mb] = v4i{};
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) f.b[s][nb] = v4i{};
    }
    // Blocks are taken two at a time (stage 0, stage 1) so each LDS stage is
    // its own object; the loop has a single exit and an odd last block is
    // peeled, which keeps the accumulators in place across iterations.
    int kb = 0;
    for (; kb + 2 <= nkb; kb += 2) {
        stage_step<S, G, WM, WN, MB, NB>(acc, f, lds0, lds1, lp, kb, nkb, wm, wn, half, l32);
        stage_step<S, G, WM, WN, MB, NB>(acc, f, lds1, lds0, lp, kb + 1, nkb, wm, wn, half, l32);
    }
    if (kb < nkb) stage_step<S, G, WM, WN, MB, NB>(acc, f, lds0, lds1, lp, kb, nkb, wm, wn, half, l32);
    mfma_pairs<true, S, G, MB, NB>(acc, f);
}

// Exact diagonal sums of one tile for one term, with the fragments read one
// block ahead (prefetch_step).
template <int S, int G, int WM, int WN, int MB, int NB>
__device__ __forceinline__ void pair_mainloop_prefetch(v16i (&acc)[G][MB][NB], uint4 *lds0, uint4 *lds1,
                                              const TermDesc &T, int m0, int n0) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
    const int wm = wave / WN;
    const int wn = wave % WN;
    const int half = lane >> 5;
    const int l32 = lane & 31;
    const int nkb = T.kblocks;

#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[g][mb][nb] = v16i{};
    if (nkb == 0) return;

    LoadPlan<S, G, WM, WN, MB, NB> lp;
    lp.init(T.A, T.B, T.a_rows_p, T.b_rows_p, m0, n0, wave, lane);
    // a previous term of this block (accumulating mode) may still read the stages
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // blocks 0 and 1 load together (one latency); the first step then finds
    // block 1 complete
    lp.issue(lds0, 0);
    if (1 < nkb) lp.issue(lds1, 1);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    Frags<S, G, MB, NB> f;
    read_stage<S, G, WM, WN, MB, NB>(f, lds0, wm, wn, half, l32);
    // Blocks are taken two at a time (stage 0, stage 1) so each LDS stage is
    // its own object; the loop has a single exit and an odd last block is
    // peeled.
    int kb = 0;
    for (; kb + 2 <= nkb; kb += 2) {
        prefetch_step<S, G, WM, WN, MB, NB>(acc, f, lds0, lds1, lp, kb, nkb, wm, wn, half, l32);
        prefetch_step<S, G, WM, WN, MB, NB>(acc, f, lds1, lds0, lp, kb + 1, nkb, wm, wn, half, l32);
    }
    if (kb < nkb) prefetch_step<S, G, WM, WN, MB, NB>(acc, f, lds0, lds1, lp, kb, nkb, wm, wn, half, l32);
}

// ---- per-tile main loop: a ring of three LDS stages ------------------------
// For waves that own one 32 x 32 block (tiles of 8 or 16 waves): step kb
//
//   waits until block kb + 1 has landed (this wave's loads: vmcnt, leaving
//   block kb + 2's loads in flight), barrier (every wave's share of block
//   kb + 1 is in LDS, and every wave has its fragments of block kb, so block
//   kb's stage is free);
//   starts the loads of block kb + 3 into block kb's stage;
//   runs AsmStep: the MFMAs of block kb from registers, each fragment
//   register refilled with block kb + 1's fragment once its last MFMA has
//   issued (one set of fragment registers), the reads waited for at its end.
//
// A block's loads have two steps to arrive instead of one: the reads inside
// AsmStep are invisible to the compiler, which therefore does not order them
// behind the direct-to-LDS loads still in flight (with compiler-visible LDS
// reads it waits for every such load first).  The barrier is the bare
// s_barrier: the waits it needs are the explicit ones above (the barrier of
// __syncthreads would first wait for every load in flight).  Reads of a
// stage only happen once its block is complete in every wave; loads into a
// stage only start once every wave has read it.
template <int S, int G, int WM, int WN, int MB, int NB, int MODE>
__host__ __device__ constexpr bool use_ring();

template <int S, int G, int WM, int WN, int MB, int NB>
struct RingAddr {
    using C = Cfg<S, G, WM, WN, MB, NB>;
    static constexpr int OA = 2 * C::BM * 16;  // bytes between the runs of consecutive A slices
    static constexpr int OB = 2 * C::BN * 16;
    // LDS byte addresses of this lane's A and B fragments of slice 0 in a stage
    __device__ __forceinline__ static unsigned a(const uint4 *stage, int wm, int half, int l32) {
        return static_cast<unsigned>(reinterpret_cast<uintptr_t>(stage + half * C::BM + wm * 32 + l32));
    }
    __device__ __forceinline__ static unsigned b(const uint4 *stage, int wn, int half, int l32) {
        return static_cast<unsigned>(reinterpret_cast<uintptr_t>(stage + 2 * S * C::BM + half * C::BN + wn * 32 + l32));
    }
};

template <int S, int G, int WM, int WN, int MB, int NB, typename F, typename LP>
__device__ __forceinline__ void ring_step(v16i (&acc)[G][MB][NB], F &cur, uint4 *fill, const uint4 *rd,
                                          const LP &lp, int kb, int nkb, int wm, int wn, int half, int l32) {
    using C = Cfg<S, G, WM, WN, MB, NB>;
    using RA = RingAddr<S, G, WM, WN, MB, NB>;
    if (kb + 1 < nkb) {
        if (kb + 2 < nkb)
            __builtin_amdgcn_s_waitcnt(C::WAIT_NEWEST);
        else
            __builtin_amdgcn_s_waitcnt(C::WAIT_ALL);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (kb + 3 < nkb) lp.issue(fill, kb + 3);
    }
    // the last step reads a stage no load is pending on; the values go unused
    AsmStep<S, G>::template run<RA::OA, RA::OB>(acc, cur, RA::a(rd, wm, half, l32), RA::b(rd, wn, half, l32));
}

template <int S, int G, int WM, int WN, int MB, int NB>
__device__ __forceinline__ void pair_mainloop_ring(v16i (&acc)[G][MB][NB], uint4 *lds0, uint4 *lds1, uint4 *lds2,
                                                   const TermDesc &T, int m0, int n0) {
    using C = Cfg<S, G, WM, WN, MB, NB>;
    using RA = RingAddr<S, G, WM, WN, MB, NB>;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
    const int wm = wave / WN;
    const int wn = wave % WN;
    const int half = lane >> 5;
    const int l32 = lane & 31;
    const int nkb = T.kblocks;

#pragma unroll
    for (int g = 0; g < G; ++g) acc[g][0][0] = v16i{};
    if (nkb == 0) return;

    LoadPlan<S, G, WM, WN, MB, NB> lp;
    lp.init(T.A, T.B, T.a_rows_p, T.b_rows_p, m0, n0, wave, lane);
    // a previous term of this block (accumulating mode) may still read the stages
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    lp.issue(lds0, 0);
    if (1 < nkb) lp.issue(lds1, 1);
    if (2 < nkb) lp.issue(lds2, 2);
    if (2 < nkb)
        __builtin_amdgcn_s_waitcnt(C::WAIT_NEWER2);
    else if (1 < nkb)
        __builtin_amdgcn_s_waitcnt(C::WAIT_NEWEST);
    else
        __builtin_amdgcn_s_waitcnt(C::WAIT_ALL);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    Frags<S, G, MB, NB> f;
    AsmStep<S, G>::template read<RA::OA, RA::OB>(f, RA::a(lds0, wm, half, l32), RA::b(lds0, wn, half, l32));
    // Blocks are taken three at a time so each stage keeps its own object;
    // the loop has a single exit and the last nkb % 3 blocks are peeled.
    int kb = 0;
    for (; kb + 3 <= nkb; kb += 3) {
        ring_step<S, G, WM, WN, MB, NB>(acc, f, lds0, lds1, lp, kb, nkb, wm, wn, half, l32);
        ring_step<S, G, WM, WN, MB, NB>(acc, f, lds1, lds2, lp, kb + 1, nkb, wm, wn, half, l32);
        ring_step<S, G, WM, WN, MB, NB>(acc, f, lds2, lds0, lp, kb + 2, nkb, wm, wn, half, l32);
    }
    if (kb < nkb) ring_step<S, G, WM, WN, MB, NB>(acc, f, lds0, lds1, lp, kb, nkb, wm, wn, half, l32);
    if (kb + 1 < nkb) ring_step<S, G, WM, WN, MB, NB>(acc, f, lds1, lds2, lp, kb + 1, nkb, wm, wn, half, l32);
    // the accumulators were last written by matrix-core instructions inside
    // asm blocks: wait states before ordinary instructions read them
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
}

template <int S, int G, int WM, int WN, int MB, int NB, typename F, typename LP>
__device__ __forceinline__ void ring_step2(v16i (&acc)[G][MB][NB], F &cur, uint4 *fill, const uint4 *rd,
                                           const LP &lp, int kb, int nkb, int wm, int wn, int half, int l32) {
    using C = Cfg<S, G, WM, WN, MB, NB>;
    using RA = RingAddr<S, G, WM, WN, MB, NB>;
    if (kb + 1 < nkb) {
        __builtin_amdgcn_s_waitcnt(C::WAIT_ALL);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (kb + 2 < nkb) lp.issue(fill, kb + 2);
    }
    AsmStep<S, G>::template run<RA::OA, RA::OB>(acc, cur, RA::a(rd, wm, half, l32), RA::b(rd, wn, half, l32));
}

// The ring's steps with two stages (loads one block ahead), for the 4-wave
// tiles where a third stage would leave room for only one workgroup per
// compute unit (S >= 7): the second resident workgroup covers the shorter
// lead.
template <int S, int G, int WM, int WN, int MB, int NB>
__device__ __forceinline__ void pair_mainloop_ring2(v16i (&acc)[G][MB][NB], uint4 *lds0, uint4 *lds1,
                                                    const TermDesc &T, int m0, int n0) {
    using C = Cfg<S, G, WM, WN, MB, NB>;
    using RA = RingAddr<S, G, WM, WN, MB, NB>;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
    const int wm = wave / WN;
    const int wn = wave % WN;
    const int half = lane >> 5;
    const int l32 = lane & 31;
    const int nkb = T.kblocks;

#pragma unroll
    for (int g = 0; g < G; ++g) acc[g][0][0] = v16i{};
    if (nkb == 0) return;

    LoadPlan<S, G, WM, WN, MB, NB> lp;
    lp.init(T.A, T.B, T.a_rows_p, T.b_rows_p, m0, n0, wave, lane);
    // a previous term of this block (accumulating mode) may still read the stages
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    lp.issue(lds0, 0);
    if (1 < nkb) lp.issue(lds1, 1);
    if (1 < nkb)
        __builtin_amdgcn_s_waitcnt(C::WAIT_NEWEST);
    else
        __builtin_amdgcn_s_waitcnt(C::WAIT_ALL);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    Frags<S, G, MB, NB> f;
    AsmStep<S, G>::template read<RA::OA, RA::OB>(f, RA::a(lds0, wm, half, l32), RA::b(lds0, wn, half, l32));
    // step kb: wait for block kb + 1 (the only load in flight), barrier,
    // loads of block kb + 2 into block kb's stage, then block kb's MFMAs with
    // block kb + 1's fragment reads
    int kb = 0;
    for (; kb + 2 <= nkb; kb += 2) {
        ring_step2<S, G, WM, WN, MB, NB>(acc, f, lds0, lds1, lp, kb, nkb, wm, wn, half, l32);
        ring_step2<S, G, WM, WN, MB, NB>(acc, f, lds1, lds0, lp, kb + 1, nkb, wm, wn, half, l32);
    }
    if (kb < nkb) ring_step2<S, G, WM, WN, MB, NB>(acc, f, lds0, lds1, lp, kb, nkb, wm, wn, half, l32);
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
}

// Registers of one wave: accumulators, fragments, the running sigma of the
// accumulating mode and about 24 for addresses and counters, within 256 per
// wave at two waves per SIMD (128 at four).  The prefetching loop holds two
// fragment sets; the ring one set plus four spare fragments.
template <int S, int G, int WM, int WN, int MB, int NB, int MODE>
__host__ __device__ constexpr int wave_budget_left(int frag_sets, int spares) {
    return (WM * WN >= 16 ? 128 : 256) -
           (16 * G * MB * NB + frag_sets * 4 * (S < G ? S : G) * (MB + NB) + 4 * spares +
            (MODE == kModeAccum ? 32 * MB * NB : 0) + 24);
}

template <int S, int G, int WM, int WN, int MB, int NB, int MODE>
__host__ __device__ constexpr bool use_prefetch() {
    return wave_budget_left<S, G, WM, WN, MB, NB, MODE>(2, 0) >= 0;
}

// The ring of three stages where its conditions hold: one 32 x 32 block per
// wave; 8 waves (the workgroup holds its compute unit alone anyway), or 4
// waves whose registers (more than 128 each) allow at most two workgroups
// per compute unit anyway and whose three stages still let two fit in LDS
// (S <= 6; from S = 7 the third stage would halve the occupancy, which
// measured slower); three stages within 156 KiB of LDS and the register
// budget (with 24 registers more in hand for the accumulating mode, whose
// term loop keeps more live: at S = G = 7 it spills without them).
template <int S, int G, int WM, int WN, int MB, int NB, int MODE>
__host__ __device__ constexpr bool use_ring() {
    return AsmStep<S, G>::available && MB == 1 && NB == 1 &&
           (WM * WN == 8 || (WM * WN == 4 && wave_budget_left<S, G, WM, WN, MB, NB, MODE>(1, 4) < 128 &&
                             6 * Cfg<S, G, WM, WN, MB, NB>::STAGE_BYTES <= 160 * 1024)) &&
           3 * Cfg<S, G, WM, WN, MB, NB>::STAGE_BYTES <= 156 * 1024 &&
           wave_budget_left<S, G, WM, WN, MB, NB, MODE>(1, 4) >= (MODE == kModeAccum ? 24 : 0);
}

// The two-stage ring: the 4-wave tiles the three-stage ring leaves out
// because a third stage would halve their occupancy (S >= 7), where the
// registers (more than 128 per wave) allow two workgroups per compute unit
// and their two stages fit in LDS twice.
template <int S, int G, int WM, int WN, int MB, int NB, int MODE>
__host__ __device__ constexpr bool use_ring2() {
    return !use_ring<S, G, WM, WN, MB, NB, MODE>() && AsmStep<S, G>::available && MB == 1 && NB == 1 &&
           WM * WN == 4 && wave_budget_left<S, G, WM, WN, MB, NB, MODE>(1, 4) < 128 &&
           4 * Cfg<S, G, WM, WN, MB, NB>::STAGE_BYTES <= 160 * 1024 &&
           wave_budget_left<S, G, WM, WN, MB, NB, MODE>(1, 4) >= (MODE == kModeAccum ? 24 : 0);
}

// Exact diagonal sums of one tile for one term, accumulated over all K blocks.
template <int S, int G, int WM, int WN, int MB, int NB, int MODE>
__device__ __forceinline__ void pair_mainloop(v16i (&acc)[G][MB][NB], uint4 *lds0, uint4 *lds1, uint4 *lds2,
                                              const TermDesc &T, int m0, int n0) {
    if constexpr (use_ring<S, G, WM, WN, MB, NB, MODE>())
        pair_mainloop_ring<S, G, WM, WN, MB, NB>(acc, lds0, lds1, lds2, T, m0, n0);
    else if constexpr (use_ring2<S, G, WM, WN, MB, NB, MODE>())
        pair_mainloop_ring2<S, G, WM, WN, MB, NB>(acc, lds0, lds1, T, m0, n0);
    else if constexpr (use_prefetch<S, G, WM, WN, MB, NB, MODE>())
        pair_mainloop_prefetch<S, G, WM, WN, MB, NB>(acc, lds0, lds1, T, m0, n0);
    else
        pair_mainloop_direct<S, G, WM, WN, MB, NB>(acc, lds0, lds1, T, m0, n0);
}

// Output elements whose recombinations the epilogue lets the scheduler
// interleave (their dependent FP64 chains overlap); a schedule barrier
// between groups keeps the registers of only one group live.
constexpr int kEpilogueGroup = 4;

// FP64 value of one output element from its diagonal sums (plus int64 carries).
template <int G>
__device__ __forceinline__ double horner(const long long (&q)[G], int32_t ei, int32_t fj) {
    if (ei == kExpBad || fj == kExpBad) return __longlong_as_double(0x7ff8000000000000ll);
    double h = static_cast<double>(q[G - 1]);
#pragma unroll
    for (int g = G - 2; g >= 0; --g) h = fma(h, 0x1p-8, static_cast<double>(q[g]));
    return ldexp(h, ei + fj - 14);
}

// Fused row maxima of a GEMM-mode output.  For one 32 x 32 block a lane
// holds 16 stored values, value r of lane l at row 8 (r / 4) + 4 (l / 32) +
// r % 4, column l % 32.  Their magnitudes, as bit patterns with the sign
// cleared (integer order is magnitude order, NaN above Inf), are reduced
// over the 32 columns by halving exchanges: each step keeps half of the rows
// and takes the partner's other half.  The epilogue visits the values in
// the order 0, 8, 1, 9, ... and makes the first exchange (partner l ^ 16)
// as soon as values q and 8 + q exist, so only 8 partial maxima stay live.
// First exchange of values q (lo) and 8 + q (hi): the partner's half.  Its
// result is used one pair later, so the exchange latency is hidden behind
// the next element's recombination.
__device__ __forceinline__ void emax_issue(long long lo, long long hi, int l32, long long &keep, long long &got) {
    const bool b4 = l32 & 16;
    got = __shfl_xor(b4 ? lo : hi, 16);
    keep = b4 ? hi : lo;
}

typedef __attribute__((address_space(1))) int32_t global_i32;

// Atomic max on global memory, through the global address space: through a
// generic pointer (which may point into LDS) the compiler first waits for
// every load into LDS in flight.
__device__ __forceinline__ void global_atomic_max(int32_t *p, int32_t v) {
    __hip_atomic_fetch_max((global_i32 *)reinterpret_cast<uintptr_t>(p), v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// The remaining exchanges (partners l ^ 8, 4, 2, 1), then the even lanes
// turn their row's maximum into an exponent code and combine it into emax
// with one atomic max.  The columns j0 .. j0 + 31 map to one emax group.
__device__ __forceinline__ void emax_block(const OutDesc &out, const long long (&w8)[8], int i0, int j0,
                                           int half, int l32) {
    const bool b4 = l32 & 16, b3 = l32 & 8, b2 = l32 & 4, b1 = l32 & 2;
    long long w4[4], w2[2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const long long t = __shfl_xor(b3 ? w8[q] : w8[4 + q], 8);
        const long long k = b3 ? w8[4 + q] : w8[q];
        w4[q] = k > t ? k : t;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const long long t = __shfl_xor(b2 ? w4[q] : w4[2 + q], 4);
        const long long k = b2 ? w4[2 + q] : w4[q];
        w2[q] = k > t ? k : t;
    }
    long long w;
    {
        const long long t = __shfl_xor(b1 ? w2[0] : w2[1], 2);
        const long long k = b1 ? w2[1] : w2[0];
        w = k > t ? k : t;
    }
    {
        const long long t = __shfl_xor(w, 1);
        w = w > t ? w : t;
    }
    // this lane's row: r = 8 b4 + 4 b3 + 2 b2 + b1
    const int r = (b4 ? 8 : 0) + (b3 ? 4 : 0) + (b2 ? 2 : 0) + (b1 ? 1 : 0);
    const int i = i0 + 8 * (r >> 2) + 4 * half + (r & 3);
    if (!(l32 & 1) && i < out.M && j0 < out.N && w != 0) {
        const int32_t code = w >= 0x7ff0000000000000ll ? kEmaxNaN : shared_exponent(__longlong_as_double(w));
        global_atomic_max(out.emax + static_cast<int64_t>(i) * out.ep + j0 / out.en, code);
    }
}

// The row exponents of one 32 x 32 block's recombination (the lane's 16
// values, rows i0 + 8 (r / 4) + r % 4), loaded together before it starts.
// Inside the recombination every value is kept apart from the next (so
// only one is live at a time), which would also wait for each of these
// loads in turn.
__device__ __forceinline__ void row_exponents(int32_t (&ei)[16], const int32_t *e, int M, int i0, bool jok) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = i0 + 8 * (r >> 2) + (r & 3);
        ei[r] = (jok && i < M) ? e[i] : 0;
    }
}

template <int S, int G, int WM, int WN, int MB, int NB, int MODE, bool EMAX = false, typename GetTerm>
__device__ __forceinline__ void pair_tile(const PairArgs &a, GetTerm get_term, int tb, int te,
                                          const OutDesc &out, int m0, int n0, uint4 *lds0,
                                          uint4 *lds1, uint4 *lds2) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave / WN;
    const int wn = wave % WN;
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
    if (MODE == kModeAccum && out.cont) {
        // continuing an earlier launch's sums: straight-line loads (outside
        // the output, of its first element; the value is then dropped)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < SIG; ++r) {
                    const int i = m0 + (wm * MB + mb) * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                    const int j = n0 + (wn * NB + nb) * 32 + l32;
                    const bool ok = i < out.M && j < out.N;
                    const double v = out.C[ok ? static_cast<int64_t>(i) * out.ldc + j : 0];
                    sig[mb][nb][r] = ok ? v : 0.0;
                }
    }

    // only the accumulating mode sums several terms into one tile
    const int tend = (MODE == kModeAccum) ? te : tb + 1;
    for (int ti = tb; ti < tend; ++ti) {
        const TermDesc T = get_term(ti);
        v16i acc[G][MB][NB];
        pair_mainloop<S, G, WM, WN, MB, NB, MODE>(acc, lds0, lds1, lds2, T, m0, n0);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int j = n0 + (wn * NB + nb) * 32 + l32;
            const bool jok = j < out.N;
            int32_t fj = 0;
            if (MODE != kModeQ && MODE != kModeQ64 && jok) fj = T.f[j];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                long long w8[8], mlo = 0, keep = 0, got = 0;
                int32_t ei[16];
                if constexpr (MODE != kModeQ && MODE != kModeQ64)
                    row_exponents(ei, T.e, out.M, m0 + (wm * MB + mb) * 32 + 4 * half, jok);
#pragma unroll
                for (int rr = 0; rr < 16; ++rr) {
                    // with the fused maxima, values q and 8 + q in turn
                    const int r = EMAX ? ((rr & 1) ? 8 + (rr >> 1) : (rr >> 1)) : rr;
                    // keep kEpilogueGroup elements' recombinations at a time in registers
                    if (rr % kEpilogueGroup == 0) __builtin_amdgcn_sched_barrier(0);
                    const int i = m0 + (wm * MB + mb) * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                    const bool ok = jok && i < out.M;
                    long long mag = 0;
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
                    } else if (ok) {
                        long long q[G];
#pragma unroll
                        for (int g = 0; g < G; ++g) q[g] = acc[g][mb][nb][r];
                        if (MODE == kModeGemm && a.Qw) {
                            const int64_t idx = static_cast<int64_t>(i) * a.qw_ld + j;
#pragma unroll
                            for (int g = 0; g < G; ++g) q[g] += a.Qw[g * a.qw_plane + idx];
                        }
                        const double c = horner<G>(q, ei[r], fj);
                        if (MODE == kModeGemm) {
                            double *p = out.C + static_cast<int64_t>(i) * out.ldc + j;
                            const double v = (a.beta == 0.0) ? T.alpha * c : fma(T.alpha, c, a.beta * *p);
                            *p = v;
                            mag = __double_as_longlong(v) & 0x7fffffffffffffffll;
                        } else {
                            sig[mb][nb][r % SIG] = fma(T.alpha, c, sig[mb][nb][r % SIG]);
                        }
                    }
                    if (EMAX && out.emax) {
                        if (rr & 1) {
                            if (rr > 1) w8[(rr >> 1) - 1] = keep > got ? keep : got;
                            emax_issue(mlo, mag, l32, keep, got);
                        } else {
                            mlo = mag;
                        }
                    }
                }
                if (EMAX && out.emax) {
                    w8[7] = keep > got ? keep : got;
                    emax_block(out, w8, m0 + (wm * MB + mb) * 32, n0 + (wn * NB + nb) * 32, half, l32);
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

// ---- streamed grouped kernel ----------------------------------------------
// A grid of resident workgroups takes the listed tiles from per-XCD counters
// (workgroup b serves queue b mod q, q = min(8, grid); queue x hands out
// the tiles x, x + q, x + 2q, ..., so a tile stays on the XCD its position
// in the list names, while the tiles of one XCD go to whichever of its
// workgroups is free first).  Each workgroup takes its next tile when it
// starts the current one and works through the terms in list order; the
// first K block of the next (tile, term) item is loaded into the free LDS
// stage during the last K block of the current one, so an item does not
// start with an empty pipeline and the epilogue runs while that load is in
// flight.  Same arithmetic as pair_tile, term by term.

// One K block, as stage_step; on the item's last block the loads started
// into `nxt` are the first block of the next item, if there is one.
template <int S, int G, int WM, int WN, int MB, int NB, typename F, typename LP>
__device__ __forceinline__ void stream_step(v16i (&acc)[G][MB][NB], F &f, const uint4 *cur, uint4 *nxt,
                                            const LP &lp, int kb, int nkb, bool has_next, const TermDesc &next,
                                            int nm0, int nn0, int wave, int lane, int wm, int wn, int half,
                                            int l32) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    F g;
    read_stage<S, G, WM, WN, MB, NB>(g, cur, wm, wn, half, l32);
    if (kb + 1 < nkb) {
        lp.issue(nxt, kb + 1);
    } else if (has_next) {
        LoadPlan<S, G, WM, WN, MB, NB, 1> np;
        np.init(next.A, next.B, next.a_rows_p, next.b_rows_p, nm0, nn0, wave, lane);
        np.issue(nxt, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    mfma_pairs<true, S, G, MB, NB>(acc, f);
    mfma_pairs<false, S, G, MB, NB>(acc, g);
    __builtin_amdgcn_sched_barrier(0);
    f = g;
}

// Exact diagonal sums of one item whose first K block is already on its way
// into `first`; the step of the last block starts the next item's first block.
template <int S, int G, int WM, int WN, int MB, int NB>
__device__ __forceinline__ void stream_mainloop(v16i (&acc)[G][MB][NB], uint4 *first, uint4 *second,
                                                const TermDesc &T, int m0, int n0, bool has_next,
                                                const TermDesc &next, int nm0, int nn0) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN;
    const int wn = wave % WN;
    const int half = lane >> 5;
    const int l32 = lane & 31;
    const int nkb = T.kblocks;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[g][mb][nb] = v16i{};
    if (nkb == 0) return;
    LoadPlan<S, G, WM, WN, MB, NB, 1> lp;
    lp.init(T.A, T.B, T.a_rows_p, T.b_rows_p, m0, n0, wave, lane);
    Frags<S, G, MB, NB> f;
#pragma unroll
    for (int s = 0; s < Frags<S, G, MB, NB>::T; ++s) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) f.a[s][mb] = v4i{};
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) f.b[s][nb] = v4i{};
    }
    int kb = 0;
    for (; kb + 2 <= nkb; kb += 2) {
        stream_step<S, G, WM, WN, MB, NB>(acc, f, first, second, lp, kb, nkb, has_next, next, nm0, nn0, wave, lane,
                                          wm, wn, half, l32);
        stream_step<S, G, WM, WN, MB, NB>(acc, f, second, first, lp, kb + 1, nkb, has_next, next, nm0, nn0, wave,
                                          lane, wm, wn, half, l32);
    }
    if (kb < nkb)
        stream_step<S, G, WM, WN, MB, NB>(acc, f, first, second, lp, kb, nkb, has_next, next, nm0, nn0, wave, lane,
                                          wm, wn, half, l32);
    mfma_pairs<true, S, G, MB, NB>(acc, f);
}

// Starts the first K block of an item that was not prefetched; the stages
// may still be read by the previous item, hence the barrier.
template <int S, int G, int WM, int WN, int MB, int NB>
__device__ __forceinline__ void stream_first_block(uint4 *stage, const TermDesc &T, int m0, int n0) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    LoadPlan<S, G, WM, WN, MB, NB, 1> lp;
    lp.init(T.A, T.B, T.a_rows_p, T.b_rows_p, m0, n0, wave, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    lp.issue(stage, 0);
}

// The next listed tile of this workgroup's queue that is not padding, or a
// value >= a.ntiles when the queue is empty.  Thread 0 takes the counter;
// the value reaches the other waves through LDS slot `slot` (two slots used
// alternately, so a slot is rewritten only after every wave has read it).
__device__ __forceinline__ int stream_take(const PairArgs &a, int *slots, int &slot) {
    const int nq = min(static_cast<int>(gridDim.x), 8);
    const int x = static_cast<int>(blockIdx.x) % nq;
    int t;
    do {
        if (threadIdx.x == 0) slots[slot] = x + nq * atomicAdd(a.queue + x, 1);
        __syncthreads();
        t = slots[slot];
        slot ^= 1;
    } while (t < a.ntiles && a.tiles[t].out < 0);
    return t;
}

// Called by every workgroup once its queue is empty: the last one to get
// here leaves the counters zeroed for the next launch.
__device__ __forceinline__ void stream_finish(const PairArgs &a) {
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(a.queue + 8, 1) == static_cast<int>(gridDim.x) - 1) {
            for (int q = 0; q <= 8; ++q) atomicExch(a.queue + q, 0);
            __threadfence();
        }
    }
}

// One past the last term of a tile: the GEMM mode has one term per tile.
template <int MODE>
__device__ __forceinline__ int stream_term_end(const TileDesc &d) {
    return MODE == kModeAccum ? d.term_end : d.term_begin + 1;
}

// The walk of one resident workgroup over its tiles and their terms.
template <int S, int G, int WM, int WN, int MB, int NB, int MODE, typename GetTerm>
__device__ __forceinline__ void stream_tiles(const PairArgs &a, GetTerm get_term, uint4 *lds0, uint4 *lds1) {
    static_assert(MODE == kModeGemm || MODE == kModeAccum, "streamed launches run the GEMM or accumulating mode");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave / WN;
    const int wn = wave % WN;
    const int half = lane >> 5;
    const int l32 = lane & 31;
    __shared__ int slots[2];
    int slot = 0;
    int t = stream_take(a, slots, slot);
    if (t >= a.ntiles) {
        stream_finish(a);
        return;
    }
    TileDesc td = a.tiles[t];
    bool pending = false;  // the current item's first block is on its way into lds0 (in0) or lds1
    bool in0 = true;
    constexpr int SIG = (MODE == kModeAccum) ? 16 : 1;
    while (true) {
        OutDesc od = a.outs[td.out];
        if (a.out_base) od.C = a.out_base + reinterpret_cast<intptr_t>(od.C);
        const int m0 = td.m0, n0 = td.n0;
        const int te = stream_term_end<MODE>(td);
        const int tn = stream_take(a, slots, slot);
        double sig[MB][NB][SIG];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < SIG; ++r) {
                    sig[mb][nb][r] = 0.0;
                    if (MODE == kModeAccum && od.cont) {
                        const int i = m0 + (wm * MB + mb) * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                        const int j = n0 + (wn * NB + nb) * 32 + l32;
                        if (i < od.M && j < od.N) sig[mb][nb][r] = od.C[static_cast<int64_t>(i) * od.ldc + j];
                    }
                }
        for (int ti = td.term_begin; ti < te; ++ti) {
            const TermDesc T = get_term(ti);
            // the next item: this tile's next term, else the next tile's first
            bool has_next = false;
            TermDesc N = T;
            int nm0 = m0, nn0 = n0;
            if (ti + 1 < te) {
                N = get_term(ti + 1);
                has_next = true;
            } else if (tn < a.ntiles) {
                const TileDesc nd = a.tiles[tn];
                if (nd.term_begin < stream_term_end<MODE>(nd)) {
                    N = get_term(nd.term_begin);
                    nm0 = nd.m0;
                    nn0 = nd.n0;
                    has_next = true;
                }
            }
            has_next = has_next && N.kblocks > 0 && T.kblocks > 0;
            if (!pending && T.kblocks > 0) {
                stream_first_block<S, G, WM, WN, MB, NB>(lds0, T, m0, n0);
                in0 = true;
            }
            v16i acc[G][MB][NB];
            if (in0)
                stream_mainloop<S, G, WM, WN, MB, NB>(acc, lds0, lds1, T, m0, n0, has_next, N, nm0, nn0);
            else
                stream_mainloop<S, G, WM, WN, MB, NB>(acc, lds1, lds0, T, m0, n0, has_next, N, nm0, nn0);
            // the next item's first block went into the stage the last step did not read
            pending = has_next;
            if (has_next && (T.kblocks & 1)) in0 = !in0;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int j = n0 + (wn * NB + nb) * 32 + l32;
                const bool jok = j < od.N;
                const int32_t fj = jok ? T.f[j] : 0;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    constexpr bool EMAX = MODE == kModeGemm;
                    long long w8[8], mlo = 0, keep = 0, got = 0;
                    int32_t ei[16];
                    row_exponents(ei, T.e, od.M, m0 + (wm * MB + mb) * 32 + 4 * half, jok);
#pragma unroll
                    for (int rr = 0; rr < 16; ++rr) {
                        const int r = EMAX ? ((rr & 1) ? 8 + (rr >> 1) : (rr >> 1)) : rr;
                        if (rr % kEpilogueGroup == 0) __builtin_amdgcn_sched_barrier(0);
                        const int i = m0 + (wm * MB + mb) * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                        long long mag = 0;
                        if (jok && i < od.M) {
                            long long q[G];
#pragma unroll
                            for (int g = 0; g < G; ++g) q[g] = acc[g][mb][nb][r];
                            const double c = horner<G>(q, ei[r], fj);
                            if (MODE == kModeGemm) {
                                double *p = od.C + static_cast<int64_t>(i) * od.ldc + j;
                                const double v = (a.beta == 0.0) ? T.alpha * c : fma(T.alpha, c, a.beta * *p);
                                *p = v;
                                mag = __double_as_longlong(v) & 0x7fffffffffffffffll;
                            } else {
                                sig[mb][nb][r % SIG] = fma(T.alpha, c, sig[mb][nb][r % SIG]);
                            }
                        }
                        if (EMAX && od.emax) {
                            if (rr & 1) {
                                if (rr > 1) w8[(rr >> 1) - 1] = keep > got ? keep : got;
                                emax_issue(mlo, mag, l32, keep, got);
                            } else {
                                mlo = mag;
                            }
                        }
                    }
                    if (EMAX && od.emax) {
                        w8[7] = keep > got ? keep : got;
                        emax_block(od, w8, m0 + (wm * MB + mb) * 32, n0 + (wn * NB + nb) * 32, half, l32);
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
                        if (i < od.M && j < od.N) od.C[static_cast<int64_t>(i) * od.ldc + j] = sig[mb][nb][r];
                    }
        }
        if (tn >= a.ntiles) break;
        t = tn;
        td = a.tiles[t];
    }
    stream_finish(a);
}

template <int S, int G, int WM, int WN, int MB, int NB, int MODE>
__global__ __launch_bounds__(64 * WM * WN) void k_pair_stream(PairArgs a) {
    using C = Cfg<S, G, WM, WN, MB, NB>;
    __shared__ uint4 lds0[C::STAGE];
    __shared__ uint4 lds1[C::STAGE];
    const TermDesc *terms = a.terms;
    stream_tiles<S, G, WM, WN, MB, NB, MODE>(a, [&](int i) { return terms[i]; }, lds0, lds1);
}

// ---- resident GEMM-mode kernel ---------------------------------------------
// For lists of short tiles (the first products of a block-sparse H_eff),
// where a workgroup per tile spends much of its life starting up: every
// workgroup of a grid that fits on the device at once takes the tiles
// tiles[wg_off[b] .. wg_off[b + 1]) of a schedule the host balanced by cost
// (no counters), in order.  The K blocks of its tiles form one stream
// through the three-stage ring: each step loads the block three positions
// ahead, of the current tile or of the next one, so a tile starts with its
// first blocks in LDS or on their way and its epilogue runs while they
// load.  Each tile's row and column exponents come into LDS with its first
// block (the epilogue issues no vector loads, whose waits would also wait
// for the next tile's blocks).  Same arithmetic as pair_tile's GEMM mode
// with beta = 0 and no int64 partial sums.

typedef __attribute__((address_space(4))) const TileDesc ConstTileDesc;
typedef __attribute__((address_space(4))) const OutDesc ConstOutDesc;
typedef __attribute__((address_space(4))) const int32_t ConstI32;

__device__ __forceinline__ TileDesc const_tile(const TileDesc *list, int i) {
    const ConstTileDesc *c = (const ConstTileDesc *)reinterpret_cast<uintptr_t>(list + i);
    TileDesc t;
    t.term_begin = c->term_begin;
    t.term_end = c->term_end;
    t.m0 = c->m0;
    t.n0 = c->n0;
    t.out = c->out;
    t.pad_ = 0;
    return t;
}

__device__ __forceinline__ OutDesc const_out(const OutDesc *list, int i) {
    const ConstOutDesc *c = (const ConstOutDesc *)reinterpret_cast<uintptr_t>(list + i);
    OutDesc o;
    o.C = c->C;
    o.ldc = c->ldc;
    o.M = c->M;
    o.N = c->N;
    o.emax = c->emax;
    o.ep = c->ep;
    o.en = c->en;
    o.cont = c->cont;
    o.pad_ = 0;
    return o;
}

__device__ __forceinline__ int32_t const_i32(const int32_t *p, int i) {
    return *(const ConstI32 *)reinterpret_cast<uintptr_t>(p + i);
}

// Whether the resident kernel is built for a tile shape: one 32 x 32 block
// per wave on the three-stage ring.
template <int S, int G, int WM, int WN, int MB, int NB>
__host__ __device__ constexpr bool resident_fits() {
    return MB == 1 && NB == 1 && use_ring<S, G, WM, WN, MB, NB, kModeGemm>();
}

// The exponents of one tile into LDS slot `ex` (BM row exponents, then BN
// column exponents): one 64-entry load per wave for the first BM / 64 + BN
// / 64 waves; entries past the output's edge are out of the buffer's range
// and left unused by the epilogue.
template <int BM, int BN>
__device__ __forceinline__ void resident_exponents(int32_t *ex, const TermDesc &T, const OutDesc &od, int m0, int n0,
                                                   int wave, int lane) {
    constexpr int NE = BM / 64, NF = BN / 64;
    if (wave < NE + NF) {
        const bool rows = wave < NE;
        const int first = rows ? m0 + wave * 64 : n0 + (wave - NE) * 64;
        const int valid = (rows ? od.M : od.N) - first;
        const int32_t *base = rows ? T.e : T.f;
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<int32_t *>(valid > 0 ? base + first : base), 0, valid > 0 ? 4 * min(valid, 64) : 0,
            kBufferDword3);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void *)(ex + wave * 64), 4, 4 * lane, 0, 0, 0);
    }
}

// One step of a resident item: as ring_step, except that the block three
// positions ahead may be the next item's (its block p - nkb, for p - nkb <
// nxt), and the last block also hands its stage on when the next item has a
// third block.
template <int S, int G, int WM, int WN, typename F, typename LP>
__device__ __forceinline__ void resident_step(v16i (&acc)[G][1][1], F &cur, uint4 *fill, const uint4 *rd,
                                              const LP &lp, const LP &np, int kb, int nkb, int nxt, int wm, int wn,
                                              int half, int l32) {
    using C = Cfg<S, G, WM, WN, 1, 1>;
    using RA = RingAddr<S, G, WM, WN, 1, 1>;
    const int p = kb + 3;
    if (kb + 1 < nkb) {
        // block kb + 1 has arrived once only the position after it may still load
        const bool ahead = kb + 2 < nkb || kb + 2 - nkb < nxt;
        if (ahead)
            __builtin_amdgcn_s_waitcnt(C::WAIT_NEWEST);
        else
            __builtin_amdgcn_s_waitcnt(C::WAIT_ALL);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (p < nkb)
            lp.issue(fill, p);
        else if (p - nkb < nxt)
            np.issue(fill, p - nkb);
    } else if (p - nkb < nxt) {
        // every wave has read this block's fragments before its stage is refilled
        __builtin_amdgcn_s_waitcnt(C::WAIT_LDS);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        np.issue(fill, p - nkb);
    }
    AsmStep<S, G>::template run<RA::OA, RA::OB>(acc, cur, RA::a(rd, wm, half, l32), RA::b(rd, wn, half, l32));
}

// The diagonal sums of one item whose first min(nkb, 3) blocks are issued
// into s0, s1, s2 (in that order) with its exponents before them; issues the
// next item's exponents (through `next_exp`) and its first `nxt` blocks.
template <int S, int G, int WM, int WN, typename LP, typename NextExp>
__device__ __forceinline__ void resident_item(v16i (&acc)[G][1][1], uint4 *s0, uint4 *s1, uint4 *s2, const LP &lp,
                                              int nkb, const LP &np, int nxt, NextExp next_exp) {
    using C = Cfg<S, G, WM, WN, 1, 1>;
    using RA = RingAddr<S, G, WM, WN, 1, 1>;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN;
    const int wn = wave % WN;
    const int half = lane >> 5;
    const int l32 = lane & 31;
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g][0][0] = v16i{};
    if (nkb == 0) {
        // no blocks: the exponents have arrived and no wave reads the stages
        __builtin_amdgcn_s_waitcnt(C::WAIT_ALL);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        next_exp();
        if (0 < nxt) np.issue(s0, 0);
        if (1 < nxt) np.issue(s1, 1);
        if (2 < nxt) np.issue(s2, 2);
        return;
    }
    // block 0 (and the exponents issued before it) has arrived, while this
    // item's blocks 1 and 2 may still load
    if (2 < nkb)
        __builtin_amdgcn_s_waitcnt(C::WAIT_NEWER2);
    else if (1 < nkb)
        __builtin_amdgcn_s_waitcnt(C::WAIT_NEWEST);
    else
        __builtin_amdgcn_s_waitcnt(C::WAIT_ALL);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    // the other exponent slot was last read by the previous item's epilogue
    next_exp();
    // positions nkb .. 2 of a short item take the next item's first blocks
    if (nkb == 1) {
        if (0 < nxt) np.issue(s1, 0);
        if (1 < nxt) np.issue(s2, 1);
    } else if (nkb == 2) {
        if (0 < nxt) np.issue(s2, 0);
    }
    Frags<S, G, 1, 1> f;
    AsmStep<S, G>::template read<RA::OA, RA::OB>(f, RA::a(s0, wm, half, l32), RA::b(s0, wn, half, l32));
    int kb = 0;
    for (; kb + 3 <= nkb; kb += 3) {
        resident_step<S, G, WM, WN>(acc, f, s0, s1, lp, np, kb, nkb, nxt, wm, wn, half, l32);
        resident_step<S, G, WM, WN>(acc, f, s1, s2, lp, np, kb + 1, nkb, nxt, wm, wn, half, l32);
        resident_step<S, G, WM, WN>(acc, f, s2, s0, lp, np, kb + 2, nkb, nxt, wm, wn, half, l32);
    }
    if (kb < nkb) resident_step<S, G, WM, WN>(acc, f, s0, s1, lp, np, kb, nkb, nxt, wm, wn, half, l32);
    if (kb + 1 < nkb) resident_step<S, G, WM, WN>(acc, f, s1, s2, lp, np, kb + 1, nkb, nxt, wm, wn, half, l32);
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
}

// The epilogue's exponents from LDS slot `ex`: the lane's 16 row exponents
// (four runs of four) and its column's, read in one asm block that waits for
// them itself.  A read the compiler sees would first wait for every load
// into LDS in flight, the next item's blocks among them.
template <int BM>
__device__ __forceinline__ void resident_read_exponents(int32_t (&ei)[16], int32_t &fj, const int32_t *ex, int wm,
                                                        int wn, int half, int l32) {
    const unsigned rows = static_cast<unsigned>(reinterpret_cast<uintptr_t>(ex + wm * 32 + 4 * half));
    const unsigned col = static_cast<unsigned>(reinterpret_cast<uintptr_t>(ex + BM + wn * 32 + l32));
    v4i q0, q1, q2, q3;
    int32_t c;
    asm volatile(
        "ds_read_b128 %0, %5\n\t"
        "ds_read_b128 %1, %5 offset:32\n\t"
        "ds_read_b128 %2, %5 offset:64\n\t"
        "ds_read_b128 %3, %5 offset:96\n\t"
        "ds_read_b32 %4, %6\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=v"(q0), "=v"(q1), "=v"(q2), "=v"(q3), "=v"(c)
        : "v"(rows), "v"(col)
        : "memory");
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ei[k] = q0[k];
        ei[4 + k] = q1[k];
        ei[8 + k] = q2[k];
        ei[12 + k] = q3[k];
    }
    fj = c;
}

// The GEMM-mode epilogue of one item (beta = 0) with its exponents from LDS.
template <int S, int G, int WM, int WN>
__device__ __forceinline__ void resident_epilogue(const OutDesc &out, const TermDesc &T, v16i (&acc)[G][1][1],
                                                  int m0, int n0, const int32_t *ex) {
    using C = Cfg<S, G, WM, WN, 1, 1>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave / WN;
    const int wn = wave % WN;
    const int half = lane >> 5;
    const int l32 = lane & 31;
    const int j = n0 + wn * 32 + l32;
    const bool jok = j < out.N;
    int32_t ei[16], fj;
    resident_read_exponents<C::BM>(ei, fj, ex, wm, wn, half, l32);
    long long w8[8], mlo = 0, keep = 0, got = 0;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        const int r = (rr & 1) ? 8 + (rr >> 1) : (rr >> 1);
        if (rr % kEpilogueGroup == 0) __builtin_amdgcn_sched_barrier(0);
        const int i = m0 + wm * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        long long mag = 0;
        if (jok && i < out.M) {
            long long q[G];
#pragma unroll
            for (int g = 0; g < G; ++g) q[g] = acc[g][0][0][r];
            const double v = T.alpha * horner<G>(q, ei[r], fj);
            out.C[static_cast<int64_t>(i) * out.ldc + j] = v;
            mag = __double_as_longlong(v) & 0x7fffffffffffffffll;
        }
        if (out.emax) {
            if (rr & 1) {
                if (rr > 1) w8[(rr >> 1) - 1] = keep > got ? keep : got;
                emax_issue(mlo, mag, l32, keep, got);
            } else {
                mlo = mag;
            }
        }
    }
    if (out.emax) {
        w8[7] = keep > got ? keep : got;
        emax_block(out, w8, m0 + wm * 32, n0 + wn * 32, half, l32);
    }
}

template <int S, int G, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_pair_resident(PairArgs a) {
    using C = Cfg<S, G, WM, WN, 1, 1>;
    using LP = LoadPlan<S, G, WM, WN, 1, 1, 2>;
    __shared__ uint4 st[3][C::STAGE];
    __shared__ __align__(16) int32_t ex[2][C::BM + C::BN];
    const int t0 = const_i32(a.wg_off, blockIdx.x), t1 = const_i32(a.wg_off, blockIdx.x + 1);
    if (t0 >= t1) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    TileDesc td = const_tile(a.tiles, t0);
    OutDesc od = const_out(a.outs, td.out);
    if (a.out_base) od.C = a.out_base + reinterpret_cast<intptr_t>(od.C);
    TermDesc T = const_term(a.terms, td.term_begin);
    LP lp;
    lp.init(T.A, T.B, T.a_rows_p, T.b_rows_p, td.m0, td.n0, wave, lane);
    resident_exponents<C::BM, C::BN>(ex[0], T, od, td.m0, td.n0, wave, lane);
    if (0 < T.kblocks) lp.issue(st[0], 0);
    if (1 < T.kblocks) lp.issue(st[1], 1);
    if (2 < T.kblocks) lp.issue(st[2], 2);
    int ph = 0;   // stage of the current item's first block
    int slot = 0; // its exponent slot
    for (int t = t0; t < t1; ++t) {
        const bool more = t + 1 < t1;
        const TileDesc nd = const_tile(a.tiles, more ? t + 1 : t);
        OutDesc nod = const_out(a.outs, nd.out);
        if (a.out_base) nod.C = a.out_base + reinterpret_cast<intptr_t>(nod.C);
        const TermDesc N = const_term(a.terms, nd.term_begin);
        LP np;
        np.init(N.A, N.B, N.a_rows_p, N.b_rows_p, nd.m0, nd.n0, wave, lane);
        const int nxt = more ? min(N.kblocks, 3) : 0;
        int32_t *nex = ex[slot ^ 1];
        v16i acc[G][1][1];
        uint4 *s0 = st[ph];
        uint4 *s1 = st[ph == 2 ? 0 : ph + 1];
        uint4 *s2 = st[ph == 0 ? 2 : ph - 1];
        resident_item<S, G, WM, WN>(acc, s0, s1, s2, lp, T.kblocks, np, nxt, [&]() {
            if (more) resident_exponents<C::BM, C::BN>(nex, N, nod, nd.m0, nd.n0, wave, lane);
        });
        resident_epilogue<S, G, WM, WN>(od, T, acc, td.m0, td.n0, ex[slot]);
        ph = (ph + T.kblocks) % 3;
        slot ^= 1;
        td = nd;
        od = nod;
        T = N;
        lp = np;
    }
}

// ---- paired-term accumulating kernel ---------------------------------------
// For term lists over few tiles (a Davidson step's sigma of 1024 x 1024 is
// 256 tiles of 64 x 64), where a workgroup of four waves per tile leaves one
// wave per SIMD and every wait of that wave idles the matrix cores: eight
// waves per tile in two groups of four, each group with its own three-stage
// ring, group g taking the tile's terms 2 r + g in round r.  The FP64 value
// of each term (the Horner recombination of its diagonal sums) goes through
// LDS, and each group adds the round's two values, in term order, into its
// half of the running sums (the lane's values 8 g .. 8 g + 7), so the sums
// are those of the one-group kernel.  Both rings of a round run as many
// steps as the longer term has K blocks (the other group's steps past its
// own blocks load and multiply nothing), so every wave meets the same
// barriers.

template <int S, int G>
__host__ __device__ constexpr bool terms2_fits() {
    return use_ring<S, G, 2, 2, 1, 1, kModeAccum>() && 6 * Cfg<S, G, 2, 2, 1, 1>::STAGE_BYTES <= 156 * 1024;
}

// One step of a group's ring: as ring_step over `nsteps` steps of which the
// first `nvalid` have blocks.
template <int S, int G, typename F, typename LP>
__device__ __forceinline__ void group_step(v16i (&acc)[G][1][1], F &cur, uint4 *fill, const uint4 *rd, const LP &lp,
                                           int kb, int nsteps, int nvalid, int wm, int wn, int half, int l32) {
    using C = Cfg<S, G, 2, 2, 1, 1>;
    using RA = RingAddr<S, G, 2, 2, 1, 1>;
    if (kb + 1 < nsteps) {
        // block kb + 1 (if any) has arrived once only block kb + 2 may still load
        if (kb + 2 < nvalid)
            __builtin_amdgcn_s_waitcnt(C::WAIT_NEWEST);
        else
            __builtin_amdgcn_s_waitcnt(C::WAIT_ALL);
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (kb + 3 < nvalid) lp.issue(fill, kb + 3);
    }
    if (kb < nvalid)
        AsmStep<S, G>::template run<RA::OA, RA::OB>(acc, cur, RA::a(rd, wm, half, l32), RA::b(rd, wn, half, l32));
}

// The diagonal sums of a group's term of `nvalid` K blocks over a round of
// `nsteps` >= nvalid steps; returns with the group's loads all arrived.
template <int S, int G, typename LP>
__device__ __forceinline__ void group_ring(v16i (&acc)[G][1][1], uint4 *s0, uint4 *s1, uint4 *s2, const LP &lp,
                                           int nvalid, int nsteps, int wm, int wn, int half, int l32) {
    using C = Cfg<S, G, 2, 2, 1, 1>;
    using RA = RingAddr<S, G, 2, 2, 1, 1>;
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g][0][0] = v16i{};
    if (nsteps == 0) return;
    // the previous round's reads of LDS (fragments, exchanged values) are done
    __builtin_amdgcn_s_waitcnt(C::WAIT_LDS);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (0 < nvalid) lp.issue(s0, 0);
    if (1 < nvalid) lp.issue(s1, 1);
    if (2 < nvalid) lp.issue(s2, 2);
    if (2 < nvalid)
        __builtin_amdgcn_s_waitcnt(C::WAIT_NEWER2);
    else if (1 < nvalid)
        __builtin_amdgcn_s_waitcnt(C::WAIT_NEWEST);
    else
        __builtin_amdgcn_s_waitcnt(C::WAIT_ALL);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    // (a group without blocks reads values it never uses)
    Frags<S, G, 1, 1> f;
    AsmStep<S, G>::template read<RA::OA, RA::OB>(f, RA::a(s0, wm, half, l32), RA::b(s0, wn, half, l32));
    int kb = 0;
    for (; kb + 3 <= nsteps; kb += 3) {
        group_step<S, G>(acc, f, s0, s1, lp, kb, nsteps, nvalid, wm, wn, half, l32);
        group_step<S, G>(acc, f, s1, s2, lp, kb + 1, nsteps, nvalid, wm, wn, half, l32);
        group_step<S, G>(acc, f, s2, s0, lp, kb + 2, nsteps, nvalid, wm, wn, half, l32);
    }
    if (kb < nsteps) group_step<S, G>(acc, f, s0, s1, lp, kb, nsteps, nvalid, wm, wn, half, l32);
    if (kb + 1 < nsteps) group_step<S, G>(acc, f, s1, s2, lp, kb + 1, nsteps, nvalid, wm, wn, half, l32);
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
}

template <int S, int G>
__global__ __launch_bounds__(512) void k_pair_terms2(PairArgs a) {
    using C = Cfg<S, G, 2, 2, 1, 1>;
    using LP = LoadPlan<S, G, 2, 2, 1, 1, 3>;
    // two rings of three stages; between rounds the first 64 KiB hold the
    // exchanged term values [group][wave][value][lane]
    constexpr int kRings = 2 * 3 * C::STAGE;
    constexpr int kExchange = 2 * 4 * 16 * 64 * 8 / 16;
    __shared__ uint4 lds[kRings > kExchange ? kRings : kExchange];
    const TileDesc td = a.tiles[blockIdx.x];
    if (td.out < 0) return;  // padding of the XCD order
    OutDesc od = a.outs[td.out];
    if (a.out_base) od.C = a.out_base + reinterpret_cast<intptr_t>(od.C);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = wave >> 2;
    const int w4 = wave & 3;
    const int wm = w4 / 2;
    const int wn = w4 % 2;
    const int half = lane >> 5;
    const int l32 = lane & 31;
    const int m0 = td.m0, n0 = td.n0;
    const int j = n0 + wn * 32 + l32;
    const bool jok = j < od.N;
    // this group's half of the tile's running sums: the lane's values 8 grp + q
    double sig[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) sig[q] = 0.0;
    if (od.cont) {
        // continuing an earlier launch's sums: straight-line loads (outside
        // the output, of its first element; the value is then dropped)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int r = 8 * grp + q;
            const int i = m0 + wm * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
            const bool ok = jok && i < od.M;
            const double v = od.C[ok ? static_cast<int64_t>(i) * od.ldc + j : 0];
            sig[q] = ok ? v : 0.0;
        }
    }
    uint4 *s0 = lds + grp * 3 * C::STAGE;
    uint4 *s1 = s0 + C::STAGE;
    uint4 *s2 = s1 + C::STAGE;
    double *xch = reinterpret_cast<double *>(lds);
    const TermDesc *terms = a.terms;
    for (int ta = td.term_begin; ta < td.term_end; ta += 2) {
        const bool hb = ta + 1 < td.term_end;
        const TermDesc Ta = const_term(terms, ta);
        const TermDesc Tb = const_term(terms, hb ? ta + 1 : ta);
        const int nka = Ta.kblocks, nkb = hb ? Tb.kblocks : 0;
        const int nsteps = nka > nkb ? nka : nkb;
        const TermDesc T = grp ? Tb : Ta;
        const int nvalid = grp ? nkb : nka;
        LP lp;
        lp.init(T.A, T.B, T.a_rows_p, T.b_rows_p, m0, n0, w4, lane);
        v16i acc[G][1][1];
        group_ring<S, G>(acc, s0, s1, s2, lp, nvalid, nsteps, wm, wn, half, l32);
        // every wave is done with the stages before they take the values
        __syncthreads();
        if (grp == 0 || hb) {
            const int32_t fj = jok ? T.f[j] : 0;
            int32_t ei[16];
            row_exponents(ei, T.e, od.M, m0 + wm * 32 + 4 * half, jok);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if (r % kEpilogueGroup == 0) __builtin_amdgcn_sched_barrier(0);
                const int i = m0 + wm * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                double c = 0.0;
                if (jok && i < od.M) {
                    long long q[G];
#pragma unroll
                    for (int g = 0; g < G; ++g) q[g] = acc[g][0][0][r];
                    c = horner<G>(q, ei[r], fj);
                }
                xch[((grp * 4 + w4) * 16 + r) * 64 + lane] = c;
            }
        }
        __syncthreads();
        // term a's value, then term b's, into this group's half
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int r = 8 * grp + q;
            const int i = m0 + wm * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
            if (jok && i < od.M) {
                sig[q] = fma(Ta.alpha, xch[(w4 * 16 + r) * 64 + lane], sig[q]);
                if (hb) sig[q] = fma(Tb.alpha, xch[((4 + w4) * 16 + r) * 64 + lane], sig[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int r = 8 * grp + q;
        const int i = m0 + wm * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        if (jok && i < od.M) od.C[static_cast<int64_t>(i) * od.ldc + j] = sig[q];
    }
}

// Tile index -> (tm, tn).  Blocks are dispatched to the 8 XCDs round robin;
// give every XCD a contiguous range of tiles, walked in groups of `group`
// tile rows, so the blocks that run together on one L2 share A and B panels.
// With ~32 blocks in flight per XCD as a x b tiles, each K block fetches
// a A slabs and b B slabs: for a BM x BN tile the fetch per tile is
// proportional to BM / b + BN / a, smallest at a / b = BN / BM.
__device__ __forceinline__ void tile_coords(int b, int tiles_m, int tiles_n, int group, int &tm, int &tn) {
    const int T = tiles_m * tiles_n;
    const int nx = 8;
    const int q = T / nx;
    const int rem = T - q * nx;
    const int x = b % nx;
    const int idx = b / nx;
    const int lin = x * q + (x < rem ? x : rem) + idx;
    const int per_group = group * tiles_n;
    const int gid = lin / per_group;
    const int first = gid * group;
    const int rows = tiles_m - first < group ? tiles_m - first : group;
    const int w = lin - gid * per_group;
    tm = first + w % rows;
    tn = w / rows;
}

template <int S, int G, int WM, int WN, int MB, int NB, int MODE>
__global__ __launch_bounds__(64 * WM * WN) void k_pair_single(PairArgs a, int tiles_m) {
    using C = Cfg<S, G, WM, WN, MB, NB>;
    __shared__ uint4 lds0[C::STAGE];
    __shared__ uint4 lds1[C::STAGE];
    __shared__ uint4 lds2[use_ring<S, G, WM, WN, MB, NB, MODE>() ? C::STAGE : 1];
    int tm, tn;
    constexpr int group = C::BM >= 2 * C::BN ? 4 : 8;
    tile_coords(blockIdx.x, tiles_m, a.tiles_n, group, tm, tn);
    const TermDesc term = a.term;
    pair_tile<S, G, WM, WN, MB, NB, MODE>(a, [&](int) { return term; }, 0, 1, a.out, tm * C::BM,
                                          tn * C::BN, lds0, lds1, lds2);
}

// One block per listed tile (the list is in the XCD order the plan builds).
template <int S, int G, int WM, int WN, int MB, int NB, int MODE>
__global__ __launch_bounds__(64 * WM * WN) void k_pair_grouped(PairArgs a) {
    using C = Cfg<S, G, WM, WN, MB, NB>;
    __shared__ uint4 lds0[C::STAGE];
    __shared__ uint4 lds1[C::STAGE];
    __shared__ uint4 lds2[use_ring<S, G, WM, WN, MB, NB, MODE>() ? C::STAGE : 1];
    const TileDesc td = a.tiles[blockIdx.x];
    if (td.out < 0) return;  // padding of the XCD order
    OutDesc od = a.outs[td.out];
    if (a.out_base) od.C = a.out_base + reinterpret_cast<intptr_t>(od.C);
    const TermDesc *terms = a.terms;
    pair_tile<S, G, WM, WN, MB, NB, MODE, MODE == kModeGemm>(a, [&](int i) { return const_term(terms, i); },
                                                            td.term_begin, td.term_end, od, td.m0, td.n0, lds0,
                                                            lds1, lds2);
}

// Per-(S, G) tile shape: as wide as the accumulators allow.
// Tile variants: WM x WN waves of MB x NB blocks of 32 x 32 outputs.
//   v  waves  wave tile  block tile  built when (registers per wave)
//   0  2x2    1x1        64 x 64     always
//   1  2x2    2x1        128 x 64    32 G <= 192
//   2  2x2    2x2        128 x 128   64 G <= 192
//   3  4x2    1x1        128 x 64    16 G <= 128 (two waves per SIMD)
//   4  2x4    1x1        64 x 128    16 G <= 128
//   5  2x4    2x1        128 x 128   32 G <= 160
//   6  4x4    1x1        128 x 128   16 G <= 64  (four waves per SIMD)
// Accumulators take 16 G MB NB registers; the budget leaves room for the
// operands, addresses and, with several waves per SIMD, their share of the
// register file.
constexpr int kNumVariants = 7;
__host__ __device__ constexpr int variant_wm(int v) { return v == 3 || v == 6 ? 4 : 2; }
__host__ __device__ constexpr int variant_wn(int v) { return v == 4 || v == 5 || v == 6 ? 4 : 2; }
__host__ __device__ constexpr int variant_mb(int v) { return v == 1 || v == 2 || v == 5 ? 2 : 1; }
__host__ __device__ constexpr int variant_nb(int v) { return v == 2 ? 2 : 1; }
__host__ __device__ constexpr bool variant_fits(int G, int v) {
    return v == 0 ? true
         : v == 1 ? 32 * G <= 192
         : v == 2 ? 64 * G <= 192
         : v == 3 || v == 4 ? 16 * G <= 128
         : v == 5 ? 32 * G <= 160
         : v == 6 ? 16 * G <= 64
         : false;
}
__host__ __device__ constexpr int variant_bm(int v) { return variant_wm(v) * variant_mb(v) * 32; }
__host__ __device__ constexpr int variant_bn(int v) { return variant_wn(v) * variant_nb(v) * 32; }
// default before tuning: the 128 x 64 four-wave tile where it fits
__host__ __device__ constexpr int default_variant(int G) { return variant_fits(G, 1) ? 1 : 0; }

template <int S, int G, int V>
hipError_t run_single_v(const PairArgs &a, int tiles_m, hipStream_t s) {
    constexpr int WM = variant_wm(V), WN = variant_wn(V), MB = variant_mb(V), NB = variant_nb(V);
    constexpr int NT = 64 * WM * WN;
    if constexpr (!variant_fits(G, V)) {
        return hipErrorInvalidValue;
    } else {
        const unsigned grid = static_cast<unsigned>(tiles_m) * static_cast<unsigned>(a.tiles_n);
        if (grid == 0) return hipSuccess;
        switch (a.mode) {
            case kModeGemm:
                hipLaunchKernelGGL((k_pair_single<S, G, WM, WN, MB, NB, kModeGemm>), dim3(grid), dim3(NT), 0, s, a, tiles_m);
                break;
            case kModeQ:
                if constexpr (V == 0) {
                    hipLaunchKernelGGL((k_pair_single<S, G, WM, WN, MB, NB, kModeQ>), dim3(grid), dim3(NT), 0, s, a, tiles_m);
                } else {
                    return hipErrorInvalidValue;
                }
                break;
            case kModeQ64:
                if constexpr (V == 0) {
                    hipLaunchKernelGGL((k_pair_single<S, G, WM, WN, MB, NB, kModeQ64>), dim3(grid), dim3(NT), 0, s, a, tiles_m);
                } else {
                    return hipErrorInvalidValue;
                }
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}

template <int S, int G, int V>
hipError_t run_grouped_v(const PairArgs &a, hipStream_t s) {
    constexpr int WM = variant_wm(V), WN = variant_wn(V), MB = variant_mb(V), NB = variant_nb(V);
    constexpr int NT = 64 * WM * WN;
    if constexpr (!variant_fits(G, V)) {
        return hipErrorInvalidValue;
    } else {
        if (a.ntiles == 0) return hipSuccess;
        if (a.terms2) {
            if constexpr (V == 0 && terms2_fits<S, G>()) {
                if (a.mode != kModeAccum) return hipErrorInvalidValue;
                hipLaunchKernelGGL((k_pair_terms2<S, G>), dim3(a.ntiles), dim3(512), 0, s, a);
                return hipGetLastError();
            } else {
                return hipErrorInvalidValue;
            }
        }
        if (a.nwg > 0) {
            if constexpr (resident_fits<S, G, WM, WN, MB, NB>()) {
                if (a.mode != kModeGemm || !a.wg_off || a.beta != 0.0 || a.Qw) return hipErrorInvalidValue;
                hipLaunchKernelGGL((k_pair_resident<S, G, WM, WN>), dim3(a.nwg), dim3(NT), 0, s, a);
                return hipGetLastError();
            } else {
                return hipErrorInvalidValue;
            }
        }
        if (a.stream_cus > 0) {
            if (!a.queue) return hipErrorInvalidValue;
            // resident workgroups only: the grid walks the list, nothing queues behind it
            int per_cu = 1;
            unsigned grid = 0;
            if (a.mode == kModeGemm) {
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pair_stream<S, G, WM, WN, MB, NB, kModeGemm>,
                                                                 NT, 0) != hipSuccess || per_cu < 1)
                    per_cu = 1;
                grid = static_cast<unsigned>(std::min<int64_t>(a.ntiles, static_cast<int64_t>(per_cu) * a.stream_cus));
                hipLaunchKernelGGL((k_pair_stream<S, G, WM, WN, MB, NB, kModeGemm>), dim3(grid), dim3(NT), 0, s, a);
            } else if (a.mode == kModeAccum) {
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pair_stream<S, G, WM, WN, MB, NB, kModeAccum>,
                                                                 NT, 0) != hipSuccess || per_cu < 1)
                    per_cu = 1;
                grid = static_cast<unsigned>(std::min<int64_t>(a.ntiles, static_cast<int64_t>(per_cu) * a.stream_cus));
                hipLaunchKernelGGL((k_pair_stream<S, G, WM, WN, MB, NB, kModeAccum>), dim3(grid), dim3(NT), 0, s, a);
            } else {
                return hipErrorInvalidValue;
            }
            return hipGetLastError();
        }
        switch (a.mode) {
            case kModeGemm:
                hipLaunchKernelGGL((k_pair_grouped<S, G, WM, WN, MB, NB, kModeGemm>), dim3(a.ntiles), dim3(NT), 0, s, a);
                break;
            case kModeAccum:
                hipLaunchKernelGGL((k_pair_grouped<S, G, WM, WN, MB, NB, kModeAccum>), dim3(a.ntiles), dim3(NT), 0, s, a);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}

template <int S, int G, int V>
int resident_per_cu_v() {
    constexpr int WM = variant_wm(V), WN = variant_wn(V), MB = variant_mb(V), NB = variant_nb(V);
    if constexpr (!variant_fits(G, V)) {
        return 0;
    } else if constexpr (!resident_fits<S, G, WM, WN, MB, NB>()) {
        return 0;
    } else {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pair_resident<S, G, WM, WN>, 64 * WM * WN, 0) !=
            hipSuccess)
            return 0;
        return n;
    }
}

template <int S, int G>
int resident_per_cu(int v) {
    switch (v) {
        case 0: return resident_per_cu_v<S, G, 0>();
        case 1: return resident_per_cu_v<S, G, 1>();
        case 2: return resident_per_cu_v<S, G, 2>();
        case 3: return resident_per_cu_v<S, G, 3>();
        case 4: return resident_per_cu_v<S, G, 4>();
        case 5: return resident_per_cu_v<S, G, 5>();
        case 6: return resident_per_cu_v<S, G, 6>();
        default: return 0;
    }
}

template <int S, int G>
hipError_t run_single(int v, const PairArgs &a, int tiles_m, hipStream_t s) {
    switch (v) {
        case 0: return run_single_v<S, G, 0>(a, tiles_m, s);
        case 1: return run_single_v<S, G, 1>(a, tiles_m, s);
        case 2: return run_single_v<S, G, 2>(a, tiles_m, s);
        case 3: return run_single_v<S, G, 3>(a, tiles_m, s);
        case 4: return run_single_v<S, G, 4>(a, tiles_m, s);
        case 5: return run_single_v<S, G, 5>(a, tiles_m, s);
        case 6: return run_single_v<S, G, 6>(a, tiles_m, s);
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
        case 4: return run_grouped_v<S, G, 4>(a, s);
        case 5: return run_grouped_v<S, G, 5>(a, s);
        case 6: return run_grouped_v<S, G, 6>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pair

// Per-S entry points (pairgemm_s<S>.hip).
#define OZ_DECLARE_PAIR_S(S_)                                                                   \
    hipError_t pair_single_s##S_(int G, int v, const PairArgs &a, int tiles_m, hipStream_t s);  \
    hipError_t pair_grouped_s##S_(int G, int v, const PairArgs &a, hipStream_t s);              \
    int pair_resident_s##S_(int G, int v);                                                      \
    bool pair_terms2_s##S_(int G);
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
    }                                                                                           \
    int pair_resident_s##S_(int G, int v) {                                                     \
        if (G == S_) return pair::resident_per_cu<S_, S_>(v);                                   \
        if (G == S_ + 1) return pair::resident_per_cu<S_, S_ + 1>(v);                           \
        if (G == 2 * S_ - 1) return pair::resident_per_cu<S_, 2 * S_ - 1>(v);                   \
        return 0;                                                                               \
    }                                                                                           \
    bool pair_terms2_s##S_(int G) {                                                             \
        if (G == S_) return pair::terms2_fits<S_, S_>();                                        \
        if (G == S_ + 1) return pair::terms2_fits<S_, S_ + 1>();                                \
        if (G == 2 * S_ - 1) return pair::terms2_fits<S_, 2 * S_ - 1>();                        \
        return false;                                                                           \
    }

}  // namespace oz
