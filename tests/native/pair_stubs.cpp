// Host-only stand-ins for the per-S pair-GEMM entry points of
// csrc/pairgemm_s{2..8}.hip, so the sanitizer build of the host code
// (tests/test_sanitizers.py) skips compiling those kernels.  The test program never
// reaches a launch; a call here reports an invalid value.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace oz {
#define OZ_STUB_PAIR_S(S_)                                                                               \
    hipError_t pair_single_s##S_(int, int, const PairArgs &, int, hipStream_t) { return hipErrorInvalidValue; } \
    hipError_t pair_grouped_s##S_(int, int, const PairArgs &, hipStream_t) { return hipErrorInvalidValue; } \
    int pair_resident_s##S_(int, int) { return 0; }                                                    \
    bool pair_terms2_s##S_(int) { return false; }
OZ_STUB_PAIR_S(2)
OZ_STUB_PAIR_S(3)
OZ_STUB_PAIR_S(4)
OZ_STUB_PAIR_S(5)
OZ_STUB_PAIR_S(6)
OZ_STUB_PAIR_S(7)
OZ_STUB_PAIR_S(8)
#undef OZ_STUB_PAIR_S
}  // namespace oz
