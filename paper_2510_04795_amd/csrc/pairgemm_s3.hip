// Pair-GEMM kernels for S = 3 slices (G = S, S + 1, 2S - 1).
#include "pairgemm_impl.h"

namespace oz {
OZ_DEFINE_PAIR_S(3)
}  // namespace oz
