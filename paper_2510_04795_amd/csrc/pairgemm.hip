// Dispatch of the pair-GEMM kernels over the slice count.
#include "pairgemm_impl.h"

namespace oz {

bool pair_supported(int S, int G) {
    if (S < 2 || S > 8) return false;
    return G == S || G == S + 1 || G == 2 * S - 1;
}

PairShape pair_shape(int S, int G) {
    PairShape sh{0, 0};
    switch (S) {
        case 2: pair_shape_s2(G, &sh); break;
        case 3: pair_shape_s3(G, &sh); break;
        case 4: pair_shape_s4(G, &sh); break;
        case 5: pair_shape_s5(G, &sh); break;
        case 6: pair_shape_s6(G, &sh); break;
        case 7: pair_shape_s7(G, &sh); break;
        case 8: pair_shape_s8(G, &sh); break;
        default: break;
    }
    return sh;
}

hipError_t launch_pair_single(int S, int G, const PairArgs &a, int tiles_m, hipStream_t s) {
    switch (S) {
        case 2: return pair_single_s2(G, a, tiles_m, s);
        case 3: return pair_single_s3(G, a, tiles_m, s);
        case 4: return pair_single_s4(G, a, tiles_m, s);
        case 5: return pair_single_s5(G, a, tiles_m, s);
        case 6: return pair_single_s6(G, a, tiles_m, s);
        case 7: return pair_single_s7(G, a, tiles_m, s);
        case 8: return pair_single_s8(G, a, tiles_m, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pair_grouped(int S, int G, const PairArgs &a, int, hipStream_t s) {
    switch (S) {
        case 2: return pair_grouped_s2(G, a, s);
        case 3: return pair_grouped_s3(G, a, s);
        case 4: return pair_grouped_s4(G, a, s);
        case 5: return pair_grouped_s5(G, a, s);
        case 6: return pair_grouped_s6(G, a, s);
        case 7: return pair_grouped_s7(G, a, s);
        case 8: return pair_grouped_s8(G, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace oz
