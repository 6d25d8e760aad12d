// Sanitizer run of the library's host code (test infrastructure): the
// csrc/*.hip files (the per-S pair-GEMM kernels replaced by pair_stubs.cpp)
// are compiled with -fsanitize=address,undefined on their host side and
// linked with this program by tests/test_sanitizers.py.  No GPU is touched: the program builds a context
// by hand and calls the entry points with arguments their checks reject
// before any HIP call (sizes, leading dimensions, slice and diagonal
// counts, block layouts and triples of an effective Hamiltonian), plus the
// pure host queries (slice rules, pair counts, workspace sizes).  Every call
// must return the expected status; the sanitizers report any out-of-bounds
// access, use after free, leak or undefined behaviour on the way.
#include <cstdio>
#include <vector>

#include "runtime.h"

static int failures = 0;
#define EXPECT(cond, what)                              \
    do {                                                \
        if (!(cond)) {                                  \
            std::fprintf(stderr, "FAIL: %s\n", what);   \
            ++failures;                                 \
        }                                               \
    } while (0)

static void queries() {
    const int bits[7] = {15, 23, 31, 39, 47, 55, 63};
    for (int S = 2; S <= 8; ++S) EXPECT(ozaki_slices_for_bits(bits[S - 2]) == S, "slices for bits");
    EXPECT(ozaki_slices_for_bits(0) == OZ_ERR_ARG, "bits 0 rejected");
    EXPECT(ozaki_pair_count(7, 13) == 49, "full mode S = 7 has 49 pairs");
    EXPECT(ozaki_pair_count(6, 0) == 21, "triangular S = 6");
    EXPECT(ozaki_pair_count(9, 0) == OZ_ERR_ARG, "S = 9 rejected");
    EXPECT(ozaki_pair_count(4, 8) == OZ_ERR_ARG, "G = 2S rejected");
    EXPECT(ozaki_max_exact_k(8, 0) == 16383, "exact K at S = 8");
    EXPECT(ozaki_dgemm_workspace_bytes(100, 100, 100, 0, 0) == 0, "native needs no workspace");
    EXPECT(ozaki_dgemm_workspace_bytes(-1, 100, 100, 6, 0) == 0, "negative size");
    EXPECT(ozaki_dgemm_workspace_bytes(2048, 2048, 2048, 8, 0) <= OZ_STATIC_WORKSPACE_BYTES,
           "n = 2048 fits the static workspace at S = 8");
    int32_t tm[16], tn[16];
    EXPECT(ozaki_pair_variants(6, 0, tm, tn, 16) > 0, "tile variants listed");
    for (int st = -6; st <= 3; ++st) EXPECT(ozaki_status_string(st) != nullptr, "status text");
}

static void gemm_arguments(ozaki_ctx ctx) {
    std::vector<double> A(64), B(64), C(64);
    EXPECT(ozaki_dgemm(nullptr, 'N', 'N', 8, 8, 8, 1.0, A.data(), 8, B.data(), 8, 0.0, C.data(), 8, 6, 0, nullptr, 0,
                       nullptr) == OZ_ERR_ARG, "NULL ctx");
    EXPECT(ozaki_dgemm(ctx, 'X', 'N', 8, 8, 8, 1.0, A.data(), 8, B.data(), 8, 0.0, C.data(), 8, 6, 0, nullptr, 0,
                       nullptr) == OZ_ERR_ARG, "transa");
    EXPECT(ozaki_dgemm(ctx, 'N', 'N', -1, 8, 8, 1.0, A.data(), 8, B.data(), 8, 0.0, C.data(), 8, 6, 0, nullptr, 0,
                       nullptr) == OZ_ERR_ARG, "negative M");
    EXPECT(ozaki_dgemm(ctx, 'N', 'N', 8, 8, 8, 1.0, A.data(), 4, B.data(), 8, 0.0, C.data(), 8, 6, 0, nullptr, 0,
                       nullptr) == OZ_ERR_ARG, "lda");
    EXPECT(ozaki_dgemm(ctx, 'N', 'T', 8, 8, 8, 1.0, A.data(), 8, B.data(), 4, 0.0, C.data(), 8, 6, 0, nullptr, 0,
                       nullptr) == OZ_ERR_ARG, "ldb");
    EXPECT(ozaki_dgemm(ctx, 'N', 'N', 8, 8, 8, 1.0, A.data(), 8, B.data(), 8, 0.0, C.data(), 7, 6, 0, nullptr, 0,
                       nullptr) == OZ_ERR_ARG, "ldc");
    EXPECT(ozaki_dgemm(ctx, 'N', 'N', 8, 8, 8, 1.0, A.data(), 8, B.data(), 8, 0.0, C.data(), 8, 9, 0, nullptr, 0,
                       nullptr) == OZ_ERR_ARG, "slices 9");
    EXPECT(ozaki_dgemm(ctx, 'N', 'N', 8, 8, 8, 1.0, A.data(), 8, B.data(), 8, 0.0, C.data(), 8, 6, 8, nullptr, 0,
                       nullptr) == OZ_ERR_ARG, "ndiag 8 for S = 6");
    EXPECT(ozaki_dgemm(ctx, 'N', 'N', 8, 8, 8, 1.0, nullptr, 8, B.data(), 8, 0.0, C.data(), 8, 6, 0, nullptr, 0,
                       nullptr) == OZ_ERR_ARG, "NULL A");
    EXPECT(ozaki_dgemm(ctx, 'N', 'N', 0, 8, 8, 1.0, A.data(), 8, B.data(), 8, 0.0, C.data(), 8, 6, 0, nullptr, 0,
                       nullptr) == OZ_OK, "empty product");
    EXPECT(ozaki_dgemm_static(ctx, 'N', 'N', 4096, 4096, 4096, 1.0, A.data(), 4096, B.data(), 4096, 0.0, C.data(),
                              4096, 6, 0, nullptr) == OZ_ERR_WORKSPACE, "static workspace too small");
}

static void heff_arguments(ozaki_ctx ctx) {
    // two left and two right sectors, phys 2; psi blocks (0,0), (1,1)
    const int32_t ld[2] = {5, 7}, rd[2] = {6, 3};
    const int32_t psi_lr[4] = {0, 0, 1, 1};
    const int64_t psi_off[2] = {0, 5 * 2 * 6};
    const int32_t L_key[6] = {0, 0, 0, 0, 1, 1};
    const int64_t L_off[2] = {0, 25};
    const int32_t R_key[6] = {0, 0, 0, 0, 1, 1};
    const int64_t R_off[2] = {0, 36};
    heff_layout lay{2, 2, 2, ld, rd, 2, psi_lr, psi_off, 2, L_key, L_off, 2, R_key, R_off};
    std::vector<double> Ld(100), Rd(100);
    heff_plan P = nullptr;
    const heff_triple good[2] = {{0, 0, 0, 0, 0, 1.0}, {0, 1, 1, 1, 1, -0.5}};
    EXPECT(heff_plan_create(nullptr, &P, &lay, Ld.data(), Rd.data(), 2, good, nullptr, 6, 0, nullptr) == OZ_ERR_ARG,
           "NULL ctx");
    EXPECT(heff_plan_create(ctx, nullptr, &lay, Ld.data(), Rd.data(), 2, good, nullptr, 6, 0, nullptr) == OZ_ERR_ARG,
           "NULL out");
    EXPECT(heff_plan_create(ctx, &P, &lay, Ld.data(), Rd.data(), 2, good, nullptr, 9, 0, nullptr) == OZ_ERR_ARG,
           "slices 9");
    const heff_triple no_L[1] = {{3, 0, 0, 0, 0, 1.0}};
    EXPECT(heff_plan_create(ctx, &P, &lay, Ld.data(), Rd.data(), 1, no_L, nullptr, 6, 0, nullptr) == OZ_ERR_ARG,
           "triple without an L block");
    const heff_triple no_sigma[1] = {{0, 0, 0, 0, 1, 1.0}};
    EXPECT(heff_plan_create(ctx, &P, &lay, Ld.data(), Rd.data(), 1, no_sigma, nullptr, 6, 0, nullptr) == OZ_ERR_ARG,
           "triple without its R block / sigma block");
    const int64_t overlap[2] = {0, 10};
    heff_layout bad = lay;
    bad.psi_offset = overlap;
    EXPECT(heff_plan_create(ctx, &P, &bad, Ld.data(), Rd.data(), 2, good, nullptr, 6, 0, nullptr) == OZ_ERR_ARG,
           "overlapping psi blocks");
    const int32_t rep[4] = {0, 0, 0, 0};
    bad = lay;
    bad.psi_lr = rep;
    EXPECT(heff_plan_create(ctx, &P, &bad, Ld.data(), Rd.data(), 2, good, nullptr, 6, 0, nullptr) == OZ_ERR_ARG,
           "repeated psi block");
    const int32_t zero_dim[2] = {5, 0};
    bad = lay;
    bad.left_dim = zero_dim;
    EXPECT(heff_plan_create(ctx, &P, &bad, Ld.data(), Rd.data(), 2, good, nullptr, 6, 0, nullptr) == OZ_ERR_ARG,
           "empty sector");
    const int32_t bad_key[6] = {0, 0, 0, 0, 1, 5};
    bad = lay;
    bad.L_key = bad_key;
    EXPECT(heff_plan_create(ctx, &P, &bad, Ld.data(), Rd.data(), 2, good, nullptr, 6, 0, nullptr) == OZ_ERR_ARG,
           "L block sector out of range");
    EXPECT(P == nullptr, "no plan on failure");
    EXPECT(heff_apply(nullptr, nullptr, nullptr, nullptr) == OZ_ERR_ARG, "apply NULL plan");
    EXPECT(heff_plan_destroy(nullptr) == OZ_OK, "destroy NULL plan");
    davidson d = nullptr;
    EXPECT(davidson_create(ctx, &d, nullptr, nullptr, nullptr, 8, 1e-8, 10, nullptr) == OZ_ERR_ARG, "davidson NULL plan");
    EXPECT(davidson_step(nullptr, nullptr, nullptr) == OZ_ERR_ARG, "davidson NULL solver");
    EXPECT(davidson_set_graphs(nullptr, 1) == OZ_ERR_ARG, "davidson_set_graphs NULL");
}

int main() {
    queries();
    ozaki_ctx_s c{};
    c.device = 0;
    c.num_cu = 256;
    static double never_read;
    c.static_ws = &never_read;  // only its presence is checked before the size test rejects the call
    for (auto &row : c.variant)
        for (auto &v : row) v = -1;
    gemm_arguments(&c);
    heff_arguments(&c);
    EXPECT(ozaki_last_error()[0] != '\0', "the last error is kept");
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host runtime sanitizer run: all checks passed\n");
    return 0;
}
