// Host-side internals shared by the runtime translation units.
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/ozaki.h"
#include "internal.h"

#include <array>
#include <map>
#include <vector>

struct ozaki_ctx_s {
    int device = 0;
    int num_cu = 0;
    uint32_t *d_flags = nullptr;  // sticky OZ_FLAG_* bits on the device
    void *scratch = nullptr;      // grow-only scratch of the debug entry points
    void *static_ws = nullptr;    // this device's copy of the static workspace (ozaki_dgemm_static)
    size_t scratch_bytes = 0;
    // tile variant of the pair GEMM per (S, G); -1 = library default
    int variant[9][16];
    bool autotune = true;  // heff plans time the variants of their grouped phases
    int heff_launch = -1;  // grouped heff phases: -1 timed choice, 0 one workgroup per tile, k > 0 streamed on k CUs,
                           // OZ_HEFF_LAUNCH_RESIDENT resident first phase, OZ_HEFF_LAUNCH_PAIRED_TERMS paired-term second
    size_t heff_budget = 0;  // bytes for a heff plan's intermediates T; 0 = kHeffDefaultBudget
    // fixed choice per grouped phase of later emulated heff plans (variant < 0:
    // timed): tile variant, order (0 XCD parts, 1 longest tile first), launch
    // (0 one workgroup per tile, k > 0 streamed on k CUs)
    int heff_fix[2][3] = {{-1, 0, 0}, {-1, 0, 0}};
    // phase timing (ozaki_ctx_set_timing)
    bool timing = false;
    std::vector<hipEvent_t> events;  // pool
    size_t next_event = 0;
    struct Rec { int phase; hipEvent_t a, b; };
    std::vector<Rec> recs;
    // performant dispatch: (transa, transb, M, N, K, S, G) -> 1 emulated, 0 native
    std::map<std::array<int64_t, 7>, int> dispatch;
};

namespace oz {

// Default device bytes for the intermediates of a heff plan (T in FP64, its
// slices and exponents): the triple list runs in chunks whose first products
// fit.  The dense two-site problem at D = 2048 (Kop = 64, phys 16) needs
// 0.9 GiB per operator pair at S = 6, so 8 GiB holds nine pairs at a time.
constexpr size_t kHeffDefaultBudget = size_t(8) << 30;

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
bool valid_sg(int S, int G);
int resolve_ndiag(int S, int ndiag);
int64_t max_exact_k(int S, int G);
size_t align256(size_t x);
int ctx_scratch(ozaki_ctx ctx, size_t bytes);

// Byte offsets inside the ozaki_dgemm workspace.
struct GemmWorkspace {
    size_t a_dig, b_dig, e, f, part, qw, total;
};
GemmWorkspace gemm_workspace(int64_t M, int64_t N, int64_t K, int S, int G);

// Phase timing: mark() records an event on s (or returns nullptr when timing
// is off or the pool is used up); phase() files the pair under a phase id.
hipEvent_t mark(ozaki_ctx ctx, hipStream_t s);
void phase(ozaki_ctx ctx, int id, hipEvent_t a, hipEvent_t b);

// Variant for (S, G) in this context (explicit choice or the default).
int ctx_variant(ozaki_ctx ctx, int S, int G);

hipError_t slice_operand(int S, bool by_rows, const double *X, int64_t ld, int64_t R, int64_t K,
                         int32_t *e, int8_t *packed, double *part, uint32_t *flag, hipStream_t s);

// Slice descriptors for a list of blocks: exponent tasks (kExpTaskRows rows
// or kExpTaskCols columns each) and slice tasks (32 groups x kSliceTaskKB
// 32-wide K blocks each).
struct SliceSet {
    std::vector<SliceBlock> blocks;
    std::vector<SliceTask> etasks, stasks;
    int64_t e_total = 0, p_total = 0;
    // column exponent tasks split into row chunks (exponents through codes)
    bool split_cols = false;

    int64_t add(int64_t x_off, int64_t ld, int64_t R, int64_t K, bool trans, int S, int64_t *e_off,
                int64_t *p_off) {
        SliceBlock b{};
        b.x_off = x_off;
        b.ld = ld;
        b.R = static_cast<int32_t>(R);
        b.K = static_cast<int32_t>(K);
        b.trans = trans ? 1 : 0;
        b.Rp = round_up(R, kRowQ);
        b.e_off = e_total;
        b.p_off = p_total;
        *e_off = b.e_off;
        *p_off = b.p_off;
        e_total += b.Rp;
        p_total += align256(static_cast<size_t>(S) * b.Rp * round_up(K, kKB));
        const int id = static_cast<int>(blocks.size());
        blocks.push_back(b);
        const int step = trans ? kExpTaskCols : kExpTaskRows;
        const int64_t chunks = (trans && split_cols) ? std::max<int64_t>(ceil_div(K, kExpColChunk), 1) : 1;
        for (int64_t g = 0; g < R; g += step)
            for (int64_t c = 0; c < chunks; ++c)
                etasks.push_back(SliceTask{id, static_cast<int32_t>(g), static_cast<int32_t>(c), 0});
        for (int64_t kb = 0; kb < ceil_div(K, kKB); kb += kSliceTaskKB)
            for (int64_t r0 = 0; r0 < b.Rp; r0 += 32)
                stasks.push_back(SliceTask{id, static_cast<int32_t>(r0), static_cast<int32_t>(kb), 0});
        return id;
    }
};

}  // namespace oz
