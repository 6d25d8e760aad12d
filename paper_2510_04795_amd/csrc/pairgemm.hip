// Dispatch of the pair-GEMM kernels over the slice count and tile variant.
#include "pairgemm_impl.h"

namespace oz {

bool pair_supported(int S, int G) {
    if (S < 2 || S > 8) return false;
    return G == S || G == S + 1 || G == 2 * S - 1;
}

int pair_num_variants() { return pair::kNumVariants; }

bool pair_variant_ok(int G, int v) { return v >= 0 && v < pair::kNumVariants && pair::variant_fits(G, v); }

int pair_default_variant(int G) { return pair::default_variant(G); }

PairShape pair_shape(int S, int G, int v) {
    (void)S;
    if (v < 0) v = pair::default_variant(G);
    return PairShape{pair::variant_bm(v), pair::variant_bn(v)};
}

hipError_t launch_pair_single(int S, int G, int v, const PairArgs &a, int tiles_m, hipStream_t s) {
    if (v < 0) v = pair::default_variant(G);
    switch (S) {
        case 2: return pair_single_s2(G, v, a, tiles_m, s);
        case 3: return pair_single_s3(G, v, a, tiles_m, s);
        case 4: return pair_single_s4(G, v, a, tiles_m, s);
        case 5: return pair_single_s5(G, v, a, tiles_m, s);
        case 6: return pair_single_s6(G, v, a, tiles_m, s);
        case 7: return pair_single_s7(G, v, a, tiles_m, s);
        case 8: return pair_single_s8(G, v, a, tiles_m, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pair_grouped(int S, int G, int v, const PairArgs &a, hipStream_t s) {
    if (v < 0) v = pair::default_variant(G);
    switch (S) {
        case 2: return pair_grouped_s2(G, v, a, s);
        case 3: return pair_grouped_s3(G, v, a, s);
        case 4: return pair_grouped_s4(G, v, a, s);
        case 5: return pair_grouped_s5(G, v, a, s);
        case 6: return pair_grouped_s6(G, v, a, s);
        case 7: return pair_grouped_s7(G, v, a, s);
        case 8: return pair_grouped_s8(G, v, a, s);
        default: return hipErrorInvalidValue;
    }
}

int pair_resident_per_cu(int S, int G, int v) {
    if (v < 0) v = pair::default_variant(G);
    switch (S) {
        case 2: return pair_resident_s2(G, v);
        case 3: return pair_resident_s3(G, v);
        case 4: return pair_resident_s4(G, v);
        case 5: return pair_resident_s5(G, v);
        case 6: return pair_resident_s6(G, v);
        case 7: return pair_resident_s7(G, v);
        case 8: return pair_resident_s8(G, v);
        default: return 0;
    }
}

bool pair_terms2_ok(int S, int G, int v) {
    if (v != 0 || !pair_supported(S, G)) return false;
    switch (S) {
        case 2: return pair_terms2_s2(G);
        case 3: return pair_terms2_s3(G);
        case 4: return pair_terms2_s4(G);
        case 5: return pair_terms2_s5(G);
        case 6: return pair_terms2_s6(G);
        case 7: return pair_terms2_s7(G);
        case 8: return pair_terms2_s8(G);
        default: return false;
    }
}

}  // namespace oz
