// C-ABI of libozaki: context, argument checking, workspace layout and the
// GEMM-level entry points.  The effective-Hamiltonian plans live in heff.hip,
// the Davidson solver in davidson.hip.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/ozaki.h"
#include "internal.h"
#include "runtime.h"

// Workspace of ozaki_dgemm_static: one copy per GPU, held until the process
// ends.  Host code never uses this name as an address: the device address of
// each GPU's copy comes from hipGetSymbolAddress (static_scratch below).
static __device__ __align__(256) unsigned char scratch[OZ_STATIC_WORKSPACE_BYTES];

namespace oz {

namespace {
thread_local std::string g_last_error;

// Device address of `scratch` per device, looked up once per device (with
// that device current) by the first ozaki_ctx_create on it.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hipError_t static_scratch(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(OZ_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool valid_sg(int S, int G) { return pair_supported(S, G); }

int resolve_ndiag(int S, int ndiag) { return ndiag == 0 ? S : ndiag; }

int64_t max_exact_k(int S, int G) {
    const int nmax = G < S ? G : S;  // most pairs on one kept diagonal
    return static_cast<int64_t>(2147483647LL / (static_cast<int64_t>(nmax) << 14));
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

GemmWorkspace gemm_workspace(int64_t M, int64_t N, int64_t K, int S, int G) {
    GemmWorkspace w{};
    if (S == 0) return w;
    const int64_t Mp = round_up(M, kRowQ), Np = round_up(N, kRowQ), Kp = round_up(K, kKB);
    size_t off = 0;
    w.a_dig = off; off += align256(static_cast<size_t>(S) * Mp * Kp);
    w.b_dig = off; off += align256(static_cast<size_t>(S) * Np * Kp);
    w.e = off; off += align256(sizeof(int32_t) * (Mp > 0 ? Mp : 1));
    w.f = off; off += align256(sizeof(int32_t) * (Np > 0 ? Np : 1));
    w.part = off; off += align256(col_exponent_scratch(K, M > N ? M : N));
    w.qw = off;
    if (K > max_exact_k(S, G)) {
        // sized for the largest tile of any variant
        const int64_t mt = round_up(M, 128), nt = round_up(N, 128);
        off += align256(sizeof(int64_t) * static_cast<size_t>(G) * mt * nt);
    }
    w.total = off;
    return w;
}

// Exponents + slices of op(X) as an operand with R rows (groups) and inner K.
// by_rows: the groups are rows of the stored matrix (stored R x K), else its
// columns (stored K x R).
hipError_t slice_operand(int S, bool by_rows, const double *X, int64_t ld, int64_t R, int64_t K,
                         int32_t *e, int8_t *packed, double *part, uint32_t *flag, hipStream_t s) {
    hipError_t err;
    if (by_rows)
        err = launch_row_exponents(X, ld, R, K, e, flag, s);
    else
        err = launch_col_exponents(X, ld, K, R, e, part, flag, s);
    if (err != hipSuccess) return err;
    return launch_slice(S, !by_rows, X, ld, R, K, e, packed, round_up(R, kRowQ), s);
}

constexpr size_t kMaxEvents = 8192;

hipEvent_t mark(ozaki_ctx ctx, hipStream_t s) {
    if (!ctx || !ctx->timing || ctx->next_event >= ctx->events.size()) return nullptr;
    hipEvent_t e = ctx->events[ctx->next_event++];
    if (hipEventRecord(e, s) != hipSuccess) return nullptr;
    return e;
}

void phase(ozaki_ctx ctx, int id, hipEvent_t a, hipEvent_t b) {
    if (a && b) ctx->recs.push_back({id, a, b});
}

int ctx_variant(ozaki_ctx ctx, int S, int G) {
    const int v = (S >= 0 && S < 9 && G >= 0 && G < 16) ? ctx->variant[S][G] : -1;
    return v >= 0 ? v : pair_default_variant(G);
}

}  // namespace oz

using namespace oz;

extern "C" {

const char *ozaki_status_string(int status) {
    switch (status) {
        case OZ_OK: return "ok";
        case OZ_CONVERGED: return "converged";
        case OZ_STAGNATED: return "stagnated";
        case OZ_MAX_ITER: return "maximum iterations reached";
        case OZ_ERR_ARG: return "invalid argument";
        case OZ_ERR_WORKSPACE: return "workspace missing or too small";
        case OZ_ERR_HIP: return "HIP runtime error";
        case OZ_ERR_UNSUPPORTED: return "unsupported";
        case OZ_ERR_STATE: return "invalid state";
        case OZ_ERR_NOMEM: return "out of memory";
        default: return "unknown status";
    }
}

const char *ozaki_last_error(void) { return g_last_error.c_str(); }

int ozaki_version(void) { return 10000; }

int ozaki_ctx_create(ozaki_ctx *out, int device) {
    if (!out) return fail(OZ_ERR_ARG, "ozaki_ctx_create: out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(OZ_ERR_HIP, "ozaki_ctx_create: no HIP device");
    if (device < 0 || device >= n) return fail(OZ_ERR_ARG, "ozaki_ctx_create: device %d of %d", device, n);
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    auto *c = new ozaki_ctx_s();
    c->device = device;
    for (auto &row : c->variant)
        for (auto &v : row) v = -1;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) {
        delete c;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    c->num_cu = prop.multiProcessorCount;
    if ((e = static_scratch(device, &c->static_ws)) != hipSuccess) {
        delete c;
        return hip_fail(e, "ozaki_ctx_create: address of the static workspace");
    }
    if ((e = hipMalloc(&c->d_flags, sizeof(uint32_t))) != hipSuccess) {
        delete c;
        return hip_fail(e, "hipMalloc(flags)");
    }
    if ((e = hipMemset(c->d_flags, 0, sizeof(uint32_t))) != hipSuccess) {
        hipFree(c->d_flags);
        delete c;
        return hip_fail(e, "hipMemset(flags)");
    }
    *out = c;
    return OZ_OK;
}

int ozaki_ctx_destroy(ozaki_ctx ctx) {
    if (!ctx) return OZ_OK;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    if (ctx->scratch) hipFree(ctx->scratch);
    if (ctx->d_flags) hipFree(ctx->d_flags);
    for (auto &ev : ctx->events) hipEventDestroy(ev);
    delete ctx;
    return OZ_OK;
}

int ozaki_ctx_flags(ozaki_ctx ctx, uint32_t *flags_out) {
    if (!ctx || !flags_out) return fail(OZ_ERR_ARG, "ozaki_ctx_flags: NULL argument");
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    uint32_t v = 0;
    if ((e = hipMemcpy(&v, ctx->d_flags, sizeof(v), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(flags)");
    if ((e = hipMemset(ctx->d_flags, 0, sizeof(uint32_t))) != hipSuccess) return hip_fail(e, "hipMemset");
    *flags_out = v;
    return OZ_OK;
}

int ozaki_ctx_set_timing(ozaki_ctx ctx, int enable) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_ctx_set_timing: ctx is NULL");
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (enable && ctx->events.empty()) {
        ctx->events.resize(kMaxEvents);
        for (auto &ev : ctx->events)
            if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    ctx->timing = enable != 0;
    return OZ_OK;
}

int ozaki_ctx_phase_times(ozaki_ctx ctx, int32_t *phase_out, double *ms, int32_t max_phases) {
    if (!ctx || (max_phases > 0 && (!phase_out || !ms)))
        return fail(OZ_ERR_ARG, "ozaki_ctx_phase_times: NULL argument");
    hipError_t e;
    int n = 0;
    for (const auto &r : ctx->recs) {
        if (n >= max_phases) break;
        if ((e = hipEventSynchronize(r.b)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float t = 0.f;
        if ((e = hipEventElapsedTime(&t, r.a, r.b)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        phase_out[n] = r.phase;
        ms[n] = t;
        ++n;
    }
    ctx->recs.clear();
    ctx->next_event = 0;
    return n;
}

int ozaki_pair_variants(int slices, int ndiag, int32_t *tile_m, int32_t *tile_n, int32_t max_variants) {
    if (slices < 2 || slices > 8) return fail(OZ_ERR_ARG, "ozaki_pair_variants: slices = %d", slices);
    const int G = resolve_ndiag(slices, ndiag);
    if (!valid_sg(slices, G)) return fail(OZ_ERR_ARG, "ozaki_pair_variants: ndiag = %d", ndiag);
    const int nv = pair_num_variants();
    for (int v = 0; v < nv && v < max_variants; ++v) {
        const bool ok = pair_variant_ok(G, v);
        const PairShape sh = pair_shape(slices, G, v);
        if (tile_m) tile_m[v] = ok ? sh.bm : 0;
        if (tile_n) tile_n[v] = ok ? sh.bn : 0;
    }
    return nv;
}

int ozaki_ctx_set_variant(ozaki_ctx ctx, int slices, int ndiag, int variant) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_ctx_set_variant: ctx is NULL");
    if (slices < 2 || slices > 8) return fail(OZ_ERR_ARG, "ozaki_ctx_set_variant: slices = %d", slices);
    const int G = resolve_ndiag(slices, ndiag);
    if (!valid_sg(slices, G)) return fail(OZ_ERR_ARG, "ozaki_ctx_set_variant: ndiag = %d", ndiag);
    if (variant >= 0 && !pair_variant_ok(G, variant))
        return fail(OZ_ERR_ARG, "ozaki_ctx_set_variant: variant %d is not built for G = %d", variant, G);
    ctx->variant[slices][G] = variant < 0 ? -1 : variant;
    return OZ_OK;
}

int ozaki_ctx_get_variant(ozaki_ctx ctx, int slices, int ndiag) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_ctx_get_variant: ctx is NULL");
    if (slices < 2 || slices > 8) return fail(OZ_ERR_ARG, "ozaki_ctx_get_variant: slices = %d", slices);
    const int G = resolve_ndiag(slices, ndiag);
    if (!valid_sg(slices, G)) return fail(OZ_ERR_ARG, "ozaki_ctx_get_variant: ndiag = %d", ndiag);
    return ctx_variant(ctx, slices, G);
}

int ozaki_ctx_set_autotune(ozaki_ctx ctx, int enable) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_ctx_set_autotune: ctx is NULL");
    ctx->autotune = enable != 0;
    return OZ_OK;
}

int ozaki_ctx_set_heff_phase(ozaki_ctx ctx, int phase, int variant, int order, int launch) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_ctx_set_heff_phase: ctx is NULL");
    if (phase < 0 || phase > 1) return fail(OZ_ERR_ARG, "ozaki_ctx_set_heff_phase: phase = %d", phase);
    if (variant >= pair_num_variants() || order < 0 || order > 2 || (launch < 0 && launch != OZ_HEFF_LAUNCH_RESIDENT && launch != OZ_HEFF_LAUNCH_PAIRED_TERMS))
        return fail(OZ_ERR_ARG, "ozaki_ctx_set_heff_phase: variant %d, order %d, launch %d", variant, order, launch);
    ctx->heff_fix[phase][0] = variant < 0 ? -1 : variant;
    ctx->heff_fix[phase][1] = order;
    ctx->heff_fix[phase][2] = launch;
    return OZ_OK;
}

int ozaki_ctx_set_heff_budget(ozaki_ctx ctx, size_t bytes) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_ctx_set_heff_budget: ctx is NULL");
    ctx->heff_budget = bytes;
    return OZ_OK;
}

int ozaki_ctx_set_heff_launch(ozaki_ctx ctx, int mode) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_ctx_set_heff_launch: ctx is NULL");
    if (mode < OZ_HEFF_LAUNCH_PAIRED_TERMS) return fail(OZ_ERR_ARG, "ozaki_ctx_set_heff_launch: mode = %d", mode);
    ctx->heff_launch = mode;
    return OZ_OK;
}

int ozaki_dgemm_tune(ozaki_ctx ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                     const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                     int64_t ldc, int slices, int ndiag, void *workspace, size_t workspace_bytes,
                     void *stream, double *ms_out) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_dgemm_tune: ctx is NULL");
    if (slices < 2 || slices > 8) return fail(OZ_ERR_ARG, "ozaki_dgemm_tune: slices = %d", slices);
    const int G = resolve_ndiag(slices, ndiag);
    if (!valid_sg(slices, G)) return fail(OZ_ERR_ARG, "ozaki_dgemm_tune: ndiag = %d", ndiag);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    hipEvent_t ev0, ev1;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&ev1)) != hipSuccess) { hipEventDestroy(ev0); return hip_fail(e, "hipEventCreate"); }
    const int saved = ctx->variant[slices][G];
    int best = -1;
    float best_ms = 0.f;
    int rc = OZ_OK;
    for (int v = 0; v < pair_num_variants(); ++v) {
        if (ms_out) ms_out[v] = -1.0;
        if (!pair_variant_ok(G, v)) continue;
        ctx->variant[slices][G] = v;
        rc = ozaki_dgemm(ctx, transa, transb, M, N, K, 1.0, A, lda, B, ldb, 0.0, C, ldc, slices, G,
                         workspace, workspace_bytes, stream);
        if (rc != OZ_OK) break;
        hipEventRecord(ev0, s);
        for (int rep = 0; rep < 3 && rc == OZ_OK; ++rep)
            rc = ozaki_dgemm(ctx, transa, transb, M, N, K, 1.0, A, lda, B, ldb, 0.0, C, ldc, slices, G,
                             workspace, workspace_bytes, stream);
        hipEventRecord(ev1, s);
        if (rc != OZ_OK) break;
        if ((e = hipEventSynchronize(ev1)) != hipSuccess) { rc = hip_fail(e, "ozaki_dgemm_tune: sync"); break; }
        float ms = 0.f;
        hipEventElapsedTime(&ms, ev0, ev1);
        ms /= 3.f;
        if (ms_out) ms_out[v] = ms;
        if (best < 0 || ms < best_ms) { best = v; best_ms = ms; }
    }
    hipEventDestroy(ev0);
    hipEventDestroy(ev1);
    ctx->variant[slices][G] = (rc == OZ_OK && best >= 0) ? best : saved;
    return rc == OZ_OK ? best : rc;
}

int ozaki_slices_for_bits(int mantissa_bits) {
    if (mantissa_bits < 1) return fail(OZ_ERR_ARG, "ozaki_slices_for_bits: bits = %d", mantissa_bits);
    return (mantissa_bits + 1 + 7) / 8;
}

int ozaki_pair_count(int slices, int ndiag) {
    if (slices < 1 || slices > 8) return fail(OZ_ERR_ARG, "slices = %d", slices);
    const int G = resolve_ndiag(slices, ndiag);
    if (G < 1 || G > 2 * slices - 1) return fail(OZ_ERR_ARG, "ndiag = %d", ndiag);
    int n = 0;
    for (int s = 0; s < slices; ++s)
        for (int t = 0; t < slices; ++t)
            if (s + t < G) ++n;
    return n;
}

int64_t ozaki_max_exact_k(int slices, int ndiag) {
    if (slices < 1 || slices > 8) return fail(OZ_ERR_ARG, "slices = %d", slices);
    const int G = resolve_ndiag(slices, ndiag);
    if (G < 1 || G > 2 * slices - 1) return fail(OZ_ERR_ARG, "ndiag = %d", ndiag);
    return max_exact_k(slices, G);
}

size_t ozaki_dgemm_workspace_bytes(int64_t M, int64_t N, int64_t K, int slices, int ndiag) {
    if (slices == 0 || M < 0 || N < 0 || K < 0) return 0;
    if (slices < 2 || slices > 8) return 0;
    return gemm_workspace(M, N, K, slices, resolve_ndiag(slices, ndiag)).total;
}

int ozaki_dgemm(ozaki_ctx ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                double beta, double *C, int64_t ldc, int slices, int ndiag, void *workspace,
                size_t workspace_bytes, void *stream) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_dgemm: ctx is NULL");
    const bool ta = (transa == 'T' || transa == 't');
    const bool tb = (transb == 'T' || transb == 't');
    if (!ta && transa != 'N' && transa != 'n') return fail(OZ_ERR_ARG, "ozaki_dgemm: transa '%c'", transa);
    if (!tb && transb != 'N' && transb != 'n') return fail(OZ_ERR_ARG, "ozaki_dgemm: transb '%c'", transb);
    if (M < 0 || N < 0 || K < 0) return fail(OZ_ERR_ARG, "ozaki_dgemm: negative size");
    if (M > INT32_MAX / 2 || N > INT32_MAX / 2 || K > INT32_MAX / 2)
        return fail(OZ_ERR_ARG, "ozaki_dgemm: dimension above 2^30");
    const int64_t a_cols = ta ? M : K, b_cols = tb ? K : N;
    if (lda < (a_cols > 1 ? a_cols : 1)) return fail(OZ_ERR_ARG, "ozaki_dgemm: lda = %lld", (long long)lda);
    if (ldb < (b_cols > 1 ? b_cols : 1)) return fail(OZ_ERR_ARG, "ozaki_dgemm: ldb = %lld", (long long)ldb);
    if (ldc < (N > 1 ? N : 1)) return fail(OZ_ERR_ARG, "ozaki_dgemm: ldc = %lld", (long long)ldc);
    if (slices != 0 && (slices < 2 || slices > 8)) return fail(OZ_ERR_ARG, "ozaki_dgemm: slices = %d", slices);
    const int G = slices ? resolve_ndiag(slices, ndiag) : 0;
    if (slices && !valid_sg(slices, G))
        return fail(OZ_ERR_ARG, "ozaki_dgemm: ndiag = %d for slices = %d (use S, S+1 or 2S-1)", ndiag, slices);
    if (slices && (round_up(M, kRowQ) > kMaxPackedRows || round_up(N, kRowQ) > kMaxPackedRows))
        return fail(OZ_ERR_ARG, "ozaki_dgemm: M or N above %lld for the emulated path", (long long)kMaxPackedRows);
    if (M == 0 || N == 0) return OZ_OK;
    if (!C) return fail(OZ_ERR_ARG, "ozaki_dgemm: C is NULL");
    if (K > 0 && (!A || !B)) return fail(OZ_ERR_ARG, "ozaki_dgemm: A or B is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");

    if (slices == 0) {
        hipEvent_t t0 = mark(ctx, s);
        Dgemm64Args a{};
        a.term = Term64{A, B, lda, ldb, static_cast<int32_t>(K), 0, alpha};
        a.out = OutDesc{C, ldc, static_cast<int32_t>(M), static_cast<int32_t>(N)};
        a.mode = kModeGemm;
        a.beta = beta;
        e = launch_dgemm_single(ta, tb, a, ctx->num_cu, s);
        phase(ctx, OZ_PHASE_FP64, t0, mark(ctx, s));
        return e == hipSuccess ? OZ_OK : hip_fail(e, "ozaki_dgemm (fp64) launch");
    }

    const GemmWorkspace w = gemm_workspace(M, N, K, slices, G);
    if (workspace_bytes < w.total || (w.total > 0 && !workspace))
        return fail(OZ_ERR_WORKSPACE, "ozaki_dgemm: workspace %zu bytes, need %zu", workspace_bytes, w.total);
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(OZ_ERR_WORKSPACE, "ozaki_dgemm: workspace not 256-byte aligned");
    char *ws = static_cast<char *>(workspace);
    int8_t *adig = reinterpret_cast<int8_t *>(ws + w.a_dig);
    int8_t *bdig = reinterpret_cast<int8_t *>(ws + w.b_dig);
    int32_t *ev = reinterpret_cast<int32_t *>(ws + w.e);
    int32_t *fv = reinterpret_cast<int32_t *>(ws + w.f);
    double *part = reinterpret_cast<double *>(ws + w.part);
    const int64_t Mp = round_up(M, kRowQ), Np = round_up(N, kRowQ), Kp = round_up(K, kKB);

    // op(A) rows are stored rows when transa = 'N'; op(B) columns are stored rows when transb = 'T'
    hipEvent_t t0 = mark(ctx, s);
    if ((e = slice_operand(slices, !ta, A, lda, M, K, ev, adig, part, ctx->d_flags, s)) != hipSuccess)
        return hip_fail(e, "ozaki_dgemm: slicing A");
    if ((e = slice_operand(slices, tb, B, ldb, N, K, fv, bdig, part, ctx->d_flags, s)) != hipSuccess)
        return hip_fail(e, "ozaki_dgemm: slicing B");

    hipEvent_t t1 = mark(ctx, s);
    phase(ctx, OZ_PHASE_SLICE, t0, t1);
    const int64_t kmax = max_exact_k(slices, G);
    // the int64 carries between K chunks are built for the 64 x 64 tile only
    const int var = K > kmax ? 0 : ctx_variant(ctx, slices, G);
    const PairShape sh = pair_shape(slices, G, var);
    PairArgs a{};
    a.tiles_n = static_cast<int32_t>(ceil_div(N, sh.bn));
    const int tiles_m = static_cast<int>(ceil_div(M, sh.bm));
    a.term = TermDesc{adig, ev, bdig, fv, Mp, Np, static_cast<int32_t>(Kp / kKB), 0, alpha};
    a.out = OutDesc{C, ldc, static_cast<int32_t>(M), static_cast<int32_t>(N)};
    a.mode = kModeGemm;
    a.beta = beta;
    if (K > kmax) {
        // exact int32 sums per K chunk, carried between chunk launches in int64
        const int64_t chunk = kmax / kKB;
        const int64_t nkb = Kp / kKB;
        a.qw_ld = static_cast<int64_t>(a.tiles_n) * sh.bn;
        a.qw_plane = a.qw_ld * static_cast<int64_t>(tiles_m) * sh.bm;
        int64_t *qw = reinterpret_cast<int64_t *>(ws + w.qw);
        for (int64_t kb0 = 0; kb0 < nkb; kb0 += chunk) {
            const int64_t n = nkb - kb0 < chunk ? nkb - kb0 : chunk;
            PairArgs c = a;
            c.term.A = adig + kb0 * 2 * slices * Mp * 16;
            c.term.B = bdig + kb0 * 2 * slices * Np * 16;
            c.term.kblocks = static_cast<int32_t>(n);
            const bool last = kb0 + n >= nkb;
            c.mode = last ? kModeGemm : kModeQ64;
            c.qw_first = kb0 == 0;
            c.Qw = qw;
            if ((e = launch_pair_single(slices, G, var, c, tiles_m, s)) != hipSuccess)
                return hip_fail(e, "ozaki_dgemm: pair GEMM launch (chunked)");
        }
        phase(ctx, OZ_PHASE_PAIR, t1, mark(ctx, s));
        return OZ_OK;
    }
    e = launch_pair_single(slices, G, var, a, tiles_m, s);
    phase(ctx, OZ_PHASE_PAIR, t1, mark(ctx, s));
    return e == hipSuccess ? OZ_OK : hip_fail(e, "ozaki_dgemm: pair GEMM launch");
}

int ozaki_dgemm_static(ozaki_ctx ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                       double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                       double beta, double *C, int64_t ldc, int slices, int ndiag, void *stream) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_dgemm_static: ctx is NULL");
    if (!ctx->static_ws) return fail(OZ_ERR_STATE, "ozaki_dgemm_static: no static workspace on this device");
    // the same checks as ozaki_dgemm decide the workspace size; anything
    // they reject is reported by ozaki_dgemm itself below
    size_t need = 0;
    if (slices >= 2 && slices <= 8 && M >= 0 && N >= 0 && K >= 0) {
        const int G = resolve_ndiag(slices, ndiag);
        if (valid_sg(slices, G)) need = gemm_workspace(M, N, K, slices, G).total;
    }
    if (need > OZ_STATIC_WORKSPACE_BYTES)
        return fail(OZ_ERR_WORKSPACE,
                    "ozaki_dgemm_static: the product needs %zu bytes of workspace, above the static %llu "
                    "(use ozaki_dgemm with a workspace of ozaki_dgemm_workspace_bytes)",
                    need, static_cast<unsigned long long>(OZ_STATIC_WORKSPACE_BYTES));
    return ozaki_dgemm(ctx, transa, transb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, slices, ndiag,
                       ctx->static_ws, OZ_STATIC_WORKSPACE_BYTES, stream);
}

int ozaki_split(ozaki_ctx ctx, int by_columns, int64_t rows, int64_t cols, const double *X,
                int64_t ld, int slices, int8_t *digits, int32_t *exps, void *stream) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_split: ctx is NULL");
    if (slices < 2 || slices > 8) return fail(OZ_ERR_ARG, "ozaki_split: slices = %d", slices);
    if (rows < 0 || cols < 0 || ld < (cols > 1 ? cols : 1)) return fail(OZ_ERR_ARG, "ozaki_split: bad shape");
    if (rows == 0 || cols == 0) return OZ_OK;
    if (!X || !digits || !exps) return fail(OZ_ERR_ARG, "ozaki_split: NULL pointer");
    const int64_t R = by_columns ? cols : rows;
    const int64_t K = by_columns ? rows : cols;
    const int64_t Rp = round_up(R, kRowQ), Kp = round_up(K, kKB);
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    const size_t need = align256(static_cast<size_t>(slices) * Rp * Kp) + col_exponent_scratch(K, R);
    int rc = ctx_scratch(ctx, need);
    if (rc != OZ_OK) return rc;
    int8_t *packed = static_cast<int8_t *>(ctx->scratch);
    double *part = reinterpret_cast<double *>(static_cast<char *>(ctx->scratch) +
                                              align256(static_cast<size_t>(slices) * Rp * Kp));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((e = slice_operand(slices, !by_columns, X, ld, R, K, exps, packed, part, ctx->d_flags, s)) != hipSuccess)
        return hip_fail(e, "ozaki_split: slicing");
    if ((e = launch_unpack(slices, packed, Rp, R, K, digits, s)) != hipSuccess)
        return hip_fail(e, "ozaki_split: unpack");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "ozaki_split: sync");
    return OZ_OK;
}

int ozaki_pair_products(ozaki_ctx ctx, int64_t M, int64_t N, int64_t K, int slices, int ndiag,
                        const int8_t *Adig, const int8_t *BTdig, int32_t *Q, void *stream) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_pair_products: ctx is NULL");
    if (slices < 2 || slices > 8) return fail(OZ_ERR_ARG, "ozaki_pair_products: slices = %d", slices);
    const int G = resolve_ndiag(slices, ndiag);
    if (!valid_sg(slices, G)) return fail(OZ_ERR_ARG, "ozaki_pair_products: ndiag = %d", ndiag);
    if (M < 0 || N < 0 || K < 0) return fail(OZ_ERR_ARG, "ozaki_pair_products: negative size");
    if (K > max_exact_k(slices, G))
        return fail(OZ_ERR_ARG, "ozaki_pair_products: K = %lld exceeds the exact int32 range %lld",
                    (long long)K, (long long)max_exact_k(slices, G));
    if (round_up(M, kRowQ) > kMaxPackedRows || round_up(N, kRowQ) > kMaxPackedRows)
        return fail(OZ_ERR_ARG, "ozaki_pair_products: M or N above %lld", (long long)kMaxPackedRows);
    if (M == 0 || N == 0) return OZ_OK;
    if (!Q || (K > 0 && (!Adig || !BTdig))) return fail(OZ_ERR_ARG, "ozaki_pair_products: NULL pointer");
    const int64_t Mp = round_up(M, kRowQ), Np = round_up(N, kRowQ), Kp = round_up(K, kKB);
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    const size_t asz = align256(static_cast<size_t>(slices) * Mp * Kp);
    const size_t bsz = align256(static_cast<size_t>(slices) * Np * Kp);
    int rc = ctx_scratch(ctx, asz + bsz + 256);
    if (rc != OZ_OK) return rc;
    int8_t *pa = static_cast<int8_t *>(ctx->scratch);
    int8_t *pb = pa + asz;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((e = launch_pack(slices, Adig, M, K, pa, Mp, s)) != hipSuccess) return hip_fail(e, "pack A");
    if ((e = launch_pack(slices, BTdig, N, K, pb, Np, s)) != hipSuccess) return hip_fail(e, "pack B");
    const int var = 0;  // the int32 diagonal-sum output is built for the 64 x 64 tile only
    const PairShape sh = pair_shape(slices, G, var);
    PairArgs a{};
    a.tiles_n = static_cast<int32_t>(ceil_div(N, sh.bn));
    a.term = TermDesc{pa, nullptr, pb, nullptr, Mp, Np, static_cast<int32_t>(Kp / kKB), 0, 1.0};
    a.out = OutDesc{nullptr, 0, static_cast<int32_t>(M), static_cast<int32_t>(N)};
    a.mode = kModeQ;
    a.Q = Q;
    if ((e = launch_pair_single(slices, G, var, a, static_cast<int>(ceil_div(M, sh.bm)), s)) != hipSuccess)
        return hip_fail(e, "ozaki_pair_products: launch");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "ozaki_pair_products: sync");
    return OZ_OK;
}

}  // extern "C"

namespace oz {
int ctx_scratch(ozaki_ctx ctx, size_t bytes) {
    if (ctx->scratch_bytes >= bytes) return OZ_OK;
    hipError_t e;
    if (ctx->scratch) {
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        hipFree(ctx->scratch);
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    if ((e = hipMalloc(&ctx->scratch, bytes)) != hipSuccess)
        return fail(OZ_ERR_NOMEM, "scratch of %zu bytes: %s", bytes, hipGetErrorString(e));
    ctx->scratch_bytes = bytes;
    return OZ_OK;
}
}  // namespace oz
