// Emulation modes around ozaki_dgemm ("Numerical procedure": a mantissa width
// given by the user or found by the library, and eager or performant use of
// emulation).  The paper used a vendor library for these and gives no rule;
// the ones here are this library's own:
//
//  * Automatic slice count.  A prediction of the relative Frobenius error of
//    the emulated product from two statistics of the operands, rho_A (root
//    mean square over rows i of op(A) of 2^e_i / rms(row i)) and rho_B (the
//    same over columns of op(B)), against a prediction of the error of a
//    native FP64 GEMM of inner length K:
//
//      emulated(S, G) = 0.75 2^-8S [ (rho_A + rho_B) / sqrt(3)
//                                 + sqrt(n_G) (sigma_d^2 / 2^14) rho_A rho_B 2^-8(G-S) ]
//      native(K)      = 0.3 u sqrt(K)
//
//    The first term is the rounding of the operands to the fixed-point grid
//    (half a step of 2^(e - 8S + 1), uniformly distributed); the second is
//    the first dropped diagonal g = G (n_G slice pairs, digits with variance
//    sigma_d^2 = 256^2 / 12), both relative to a product of random signs.
//    The factors 0.75 and 0.3 were fitted to measured errors (measured over
//    predicted 0.63 .. 0.82 for S = 4 .. 7 at n = 256 .. 8192; 0.3 u sqrt(K)
//    within 10 % of the native GEMM's error at K = 512 .. 8192).  The choice is the (S, G), S in
//    [2, 8], G in {S, S + 1}, with the fewest slice pairs whose prediction
//    does not exceed the native one, else (8, 9); (2, 2) when an operand is
//    all zeros, (7, 7) when one holds NaN/Inf.
//
//  * Performant dispatch.  The first call of a shape with beta = 0 times the
//    native FP64 GEMM and the emulated one on its own output and remembers
//    the faster for the context; until then the emulated path is used.
#include <cmath>
#include <cstdio>

#include "runtime.h"

using namespace oz;

namespace oz {

// Statistics of one operand: exponents and sums of squares of its groups,
// copied to the host.
struct GroupStats {
    std::vector<int32_t> e;
    std::vector<double> ss;
};

namespace {

size_t stats_bytes(int64_t M, int64_t N, int64_t K) {
    const int64_t R = M > N ? M : N;
    return align256(sizeof(int32_t) * (R > 0 ? R : 1)) + align256(sizeof(double) * (R > 0 ? R : 1)) +
           align256(col_exponent_scratch(K, R > 0 ? R : 1));
}

int group_stats(ozaki_ctx ctx, bool by_rows, const double *X, int64_t ld, int64_t R, int64_t K, char *ws,
                hipStream_t s, GroupStats *out) {
    int32_t *e = reinterpret_cast<int32_t *>(ws);
    double *ss = reinterpret_cast<double *>(ws + align256(sizeof(int32_t) * (R > 0 ? R : 1)));
    double *part = reinterpret_cast<double *>(reinterpret_cast<char *>(ss) + align256(sizeof(double) * (R > 0 ? R : 1)));
    hipError_t err = by_rows ? launch_row_exponents(X, ld, R, K, e, ctx->d_flags, s)
                             : launch_col_exponents(X, ld, K, R, e, part, ctx->d_flags, s);
    if (err == hipSuccess) err = launch_group_sumsq(by_rows, X, ld, R, K, ss, part, s);
    if (err != hipSuccess) return hip_fail(err, "ozaki_choose_slices: statistics");
    out->e.resize(static_cast<size_t>(R));
    out->ss.resize(static_cast<size_t>(R));
    if ((err = hipMemcpyAsync(out->e.data(), e, sizeof(int32_t) * R, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (err = hipMemcpyAsync(out->ss.data(), ss, sizeof(double) * R, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (err = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(err, "ozaki_choose_slices: copy");
    return OZ_OK;
}

// Root mean square of 2^e / rms(group) over the groups with a nonzero sum of
// squares (0 when there are none; NaN when an exponent marks NaN/Inf).
double rho(const GroupStats &g, int64_t K) {
    double acc = 0.0;
    int64_t n = 0;
    for (size_t i = 0; i < g.e.size(); ++i) {
        if (g.e[i] == kExpBad || !std::isfinite(g.ss[i])) return NAN;
        if (!(g.ss[i] > 0.0)) continue;
        // (2^e / sqrt(ss / K))^2 in the log domain
        acc += std::exp2(2.0 * g.e[i] - std::log2(g.ss[i]) + std::log2(static_cast<double>(K)));
        ++n;
    }
    return n ? std::sqrt(acc / static_cast<double>(n)) : 0.0;
}

int pairs_on_diagonal(int S, int g) {
    int n = 0;
    for (int s = 0; s < S; ++s)
        if (g - s >= 0 && g - s < S) ++n;
    return n;
}

}  // namespace

double predicted_emulated_error(int S, int G, double rho_a, double rho_b) {
    const double sig2 = 256.0 * 256.0 / 12.0;
    const double rep = (rho_a + rho_b) / std::sqrt(3.0);
    const double trunc = std::sqrt(static_cast<double>(pairs_on_diagonal(S, G))) * (sig2 / 16384.0) * rho_a * rho_b *
                         std::exp2(-8.0 * (G - S));
    return 0.75 * std::exp2(-8.0 * S) * (rep + trunc);
}

double predicted_native_error(int64_t K) { return 0.3 * std::exp2(-53.0) * std::sqrt(static_cast<double>(K > 1 ? K : 1)); }

void choose_slices(double rho_a, double rho_b, int64_t K, int *S_out, int *G_out) {
    if (!std::isfinite(rho_a) || !std::isfinite(rho_b)) {
        *S_out = 7;
        *G_out = 7;
        return;
    }
    if (rho_a == 0.0 || rho_b == 0.0) {
        // an operand of zeros: the product is exactly zero at any width
        *S_out = 2;
        *G_out = 2;
        return;
    }
    const double target = predicted_native_error(K);
    int bestS = 8, bestG = 9, bestP = 1 << 30;
    for (int S = 2; S <= 8; ++S)
        for (int G = S; G <= S + 1; ++G) {
            if (predicted_emulated_error(S, G, rho_a, rho_b) > target) continue;
            int P = 0;
            for (int g = 0; g < G; ++g) P += pairs_on_diagonal(S, g);
            if (P < bestP) {
                bestP = P;
                bestS = S;
                bestG = G;
            }
        }
    *S_out = bestS;
    *G_out = bestG;
}

}  // namespace oz

extern "C" {

size_t ozaki_dgemm_auto_workspace_bytes(int64_t M, int64_t N, int64_t K) {
    if (M < 0 || N < 0 || K < 0) return 0;
    size_t w = stats_bytes(M, N, K) * 2;
    for (int S = 2; S <= 8; ++S)
        for (int G = S; G <= S + 1; ++G) {
            const size_t t = gemm_workspace(M, N, K, S, G).total;
            if (t > w) w = t;
        }
    return w;
}

int ozaki_choose_slices(ozaki_ctx ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                        const double *A, int64_t lda, const double *B, int64_t ldb, void *workspace,
                        size_t workspace_bytes, void *stream, int32_t *slices_out, int32_t *ndiag_out,
                        double *stats_out) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_choose_slices: ctx is NULL");
    const bool ta = transa == 'T' || transa == 't', tb = transb == 'T' || transb == 't';
    if (!ta && !(transa == 'N' || transa == 'n')) return fail(OZ_ERR_ARG, "ozaki_choose_slices: transa");
    if (!tb && !(transb == 'N' || transb == 'n')) return fail(OZ_ERR_ARG, "ozaki_choose_slices: transb");
    if (M < 0 || N < 0 || K < 0) return fail(OZ_ERR_ARG, "ozaki_choose_slices: negative size");
    const int64_t a_cols = ta ? M : K, b_cols = tb ? K : N;
    if (lda < (a_cols > 1 ? a_cols : 1)) return fail(OZ_ERR_ARG, "ozaki_choose_slices: lda");
    if (ldb < (b_cols > 1 ? b_cols : 1)) return fail(OZ_ERR_ARG, "ozaki_choose_slices: ldb");
    const size_t need = stats_bytes(M, N, K) * 2;
    if (workspace_bytes < need || !workspace)
        return fail(OZ_ERR_WORKSPACE, "ozaki_choose_slices: workspace %zu bytes, need %zu", workspace_bytes, need);
    double ra = 0.0, rb = 0.0;
    if (M > 0 && N > 0 && K > 0) {
        if (!A || !B) return fail(OZ_ERR_ARG, "ozaki_choose_slices: A or B is NULL");
        hipError_t e;
        if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
        hipStream_t s = static_cast<hipStream_t>(stream);
        char *ws = static_cast<char *>(workspace);
        GroupStats ga, gb;
        int rc;
        // op(A) rows are stored rows when transa = 'N'; op(B) columns are stored rows when transb = 'T'
        if ((rc = group_stats(ctx, !ta, A, lda, M, K, ws, s, &ga)) != OZ_OK) return rc;
        if ((rc = group_stats(ctx, tb, B, ldb, N, K, ws + stats_bytes(M, N, K), s, &gb)) != OZ_OK) return rc;
        ra = rho(ga, K);
        rb = rho(gb, K);
    }
    int S, G;
    choose_slices(ra, rb, K, &S, &G);
    if (slices_out) *slices_out = S;
    if (ndiag_out) *ndiag_out = G;
    if (stats_out) {
        stats_out[0] = ra;
        stats_out[1] = rb;
        stats_out[2] = predicted_emulated_error(S, G, ra, rb);
        stats_out[3] = predicted_native_error(K);
    }
    return OZ_OK;
}

int ozaki_dgemm_auto(ozaki_ctx ctx, char transa, char transb, int64_t M, int64_t N, int64_t K, double alpha,
                     const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C,
                     int64_t ldc, int bits, int performant, void *workspace, size_t workspace_bytes,
                     void *stream, int32_t *slices_out, int32_t *ndiag_out) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_dgemm_auto: ctx is NULL");
    if (bits < 0) return fail(OZ_ERR_ARG, "ozaki_dgemm_auto: bits = %d", bits);
    if (performant != 0 && performant != 1) return fail(OZ_ERR_ARG, "ozaki_dgemm_auto: performant = %d", performant);
    const size_t need = ozaki_dgemm_auto_workspace_bytes(M, N, K);
    if (M < 0 || N < 0 || K < 0) return fail(OZ_ERR_ARG, "ozaki_dgemm_auto: negative size");
    if (workspace_bytes < need || (need > 0 && !workspace))
        return fail(OZ_ERR_WORKSPACE, "ozaki_dgemm_auto: workspace %zu bytes, need %zu", workspace_bytes, need);
    int S, G;
    int rc;
    if (bits > 0) {
        S = (bits + 1 + 7) / 8;
        S = S < 2 ? 2 : (S > 8 ? 8 : S);
        G = S;
    } else {
        int32_t s32, g32;
        if ((rc = ozaki_choose_slices(ctx, transa, transb, M, N, K, A, lda, B, ldb, workspace, workspace_bytes, stream,
                                      &s32, &g32, nullptr)) != OZ_OK)
            return rc;
        S = s32;
        G = g32;
    }
    int use = S;  // slices of the path taken; 0 = native FP64
    if (performant && M > 0 && N > 0 && K > 0) {
        const std::array<int64_t, 7> key{transa == 't' || transa == 'T', transb == 't' || transb == 'T', M, N, K, S, G};
        auto it = ctx->dispatch.find(key);
        if (it != ctx->dispatch.end()) {
            use = it->second ? S : 0;
        } else if (beta == 0.0) {
            hipStream_t s = static_cast<hipStream_t>(stream);
            hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
            hipError_t e = hipSuccess;
            for (auto &x : ev)
                if (e == hipSuccess) e = hipEventCreate(&x);
            if (e != hipSuccess) {
                for (auto &x : ev)
                    if (x) hipEventDestroy(x);
                return hip_fail(e, "ozaki_dgemm_auto: events");
            }
            float ms_native = 0.f, ms_emul = 0.f;
            // warm both, then time one call of each
            rc = ozaki_dgemm(ctx, transa, transb, M, N, K, alpha, A, lda, B, ldb, 0.0, C, ldc, 0, 0, workspace,
                             workspace_bytes, stream);
            if (rc == OZ_OK)
                rc = ozaki_dgemm(ctx, transa, transb, M, N, K, alpha, A, lda, B, ldb, 0.0, C, ldc, S, G, workspace,
                                 workspace_bytes, stream);
            if (rc == OZ_OK) {
                hipEventRecord(ev[0], s);
                rc = ozaki_dgemm(ctx, transa, transb, M, N, K, alpha, A, lda, B, ldb, 0.0, C, ldc, 0, 0, workspace,
                                 workspace_bytes, stream);
                hipEventRecord(ev[1], s);
            }
            if (rc == OZ_OK) {
                rc = ozaki_dgemm(ctx, transa, transb, M, N, K, alpha, A, lda, B, ldb, 0.0, C, ldc, S, G, workspace,
                                 workspace_bytes, stream);
                hipEventRecord(ev[2], s);
            }
            if (rc == OZ_OK && (e = hipEventSynchronize(ev[2])) != hipSuccess) rc = hip_fail(e, "ozaki_dgemm_auto: sync");
            if (rc == OZ_OK) {
                hipEventElapsedTime(&ms_native, ev[0], ev[1]);
                hipEventElapsedTime(&ms_emul, ev[1], ev[2]);
                ctx->dispatch[key] = ms_emul < ms_native ? 1 : 0;
                use = ms_emul < ms_native ? S : 0;
            }
            for (auto &x : ev) hipEventDestroy(x);
            if (rc != OZ_OK) return rc;
        }
    }
    if (slices_out) *slices_out = use;
    if (ndiag_out) *ndiag_out = use ? G : 0;
    return ozaki_dgemm(ctx, transa, transb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, use, use ? G : 0, workspace,
                       workspace_bytes, stream);
}

}  // extern "C"
