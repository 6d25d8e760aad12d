// The two DMRG steps next to the H_eff diagonalisation: the eigenvalue
// decomposition of the reduced density matrix (truncation to the dominant
// eigenvectors) and the renormalisation of block operators into the kept
// basis.  The paper (numerical-stability discussion) runs both with native
// and with emulated FP64 linear algebra and finds the eigensolver's
// arithmetic decisive at low slice counts; both here take (slices, ndiag)
// like ozaki_dgemm, slices = 0 meaning native FP64.
//
// rdm_eig: two-sided block Jacobi on a symmetric A.  M = W A W^T with W
// orthogonal (W = I at the start; rows are the basis vectors).  The n rows
// (padded to np, a multiple of 64, with zero rows and columns) form np/32
// blocks of 32; a sweep pairs every block with every other once (round-robin
// "circle" schedule, np/32 - 1 rounds).  In a round the paired blocks sit
// next to each other, so pair k owns rows and columns [64k, 64k + 64):
//   1. eigenvectors of each pair's diagonal 64 x 64 block of M by cyclic
//      Jacobi in LDS (one workgroup per pair; one sweep unless the block
//      is already diagonal), accumulated from the identity, in that order:
//      Q_k^T (sorting them by eigenvalue would make the block rotation a
//      near-permutation between the two blocks, and block Jacobi then stalls);
//   2. R = Q^T M (rows of each pair), a grouped GEMM of inner length 64;
//   3. M' = Q^T R^T (= Q^T M Q, M symmetric), the same GEMM on R^T;
//   4. W <- Q^T W;
//   5. rows and columns move to the next round's slots (copies).
// The GEMMs of steps 2-4 run in the plan's arithmetic; step 1 in FP64.  The
// largest off-diagonal |M_rc| met in step 1 over a sweep measures
// convergence against tol |A|_F (absolute accuracy, as a tridiagonal-based
// solver gives).  The eigenvalues are then M_cc / |w_c|^2 and the
// eigenvectors the rows of W.  Padding rows and columns stay exactly zero (a
// zero entry gives an exact identity rotation), so the padding basis vectors
// are recognised by their zero restriction to the first n coordinates.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "runtime.h"

using namespace oz;

namespace {

constexpr int kBlk = 32;    // rows per Jacobi block
constexpr int kPair = 64;   // rows per pair of blocks
constexpr int kLdE = 65;    // LDS row stride of the 64 x 64 pair problems
constexpr int64_t kMaxEigN = 8192;
constexpr int kScanBlocks = 1024;
constexpr int kInnerSweeps = 1;

// Round-robin schedule of the 64 rows of a pair problem: row 63 fixed, the
// others rotate; step `step` pairs (63, step) and (step + t, step - t) mod 63.
__device__ __forceinline__ void circle_pair(int step, int t, int *p, int *q) {
    int a, b;
    if (t == 0) {
        a = 63;
        b = step;
    } else {
        a = (step + t) % 63;
        b = (step + 63 - t) % 63;
    }
    *p = a < b ? a : b;
    *q = a < b ? b : a;
}

// Block sum of v over the 256 threads, returned to all of them.
__device__ double block_sum(double v, double *red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Off-diagonal entries a_rc, r != c.  An entry is "exempt" when both
// diagonal entries are below theta (rows outside the wanted part of the
// spectrum).  Returns the largest |a_rc| of the other entries to all
// threads; with sums set also the sum of squares of the counted entries
// (sums[0]) and of the exempt ones (sums[1]).
__device__ double offdiag(const double *a, double *red, double theta, double *sums = nullptr) {
    const int tid = threadIdx.x;
    double m = 0.0, q = 0.0, qx = 0.0;
    for (int idx = tid; idx < kPair * kPair; idx += 256) {
        const int r = idx >> 6, c = idx & 63;
        if (r == c) continue;
        const double x = fabs(a[r * kLdE + c]);
        if (a[r * kLdE + r] < theta && a[c * kLdE + c] < theta) {
            qx = fma(x, x, qx);
        } else {
            m = fmax(m, x);
            q = fma(x, x, q);
        }
    }
    red[tid] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    if (sums) {
        sums[0] = block_sum(q, red);
        sums[1] = block_sum(qx, red);
    }
    return r;
}

__device__ __forceinline__ double lane_value(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// Step 1: one workgroup per pair k.  The pair's diagonal block of M (upper
// triangle, mirrored) is diagonalised by cyclic Jacobi until its largest
// off-diagonal entry is <= inner_tol or after kInnerSweeps sweeps; Qt rows
// [64k, 64k + 64) receive the accumulated rotations (row t: column t of
// their product); off_out[3k .. 3k + 2]: the block's largest counted
// off-diagonal |entry| and the sums of squares of the counted and of the
// exempt entries (both diagonals below theta) before the rotations.
// Each of the 4 waves owns 8 of a step's 32 disjoint rotations (t = wave +
// 4 i): lane i < 8 computes rotation i, readlane hands it to the wave, the
// lanes then sweep the 64 columns (row pass) and the 64 rows (column pass).
__global__ __launch_bounds__(256) void k_pair_eig(const double *__restrict__ M, int64_t ldm,
                                                  double *__restrict__ Qt, double *__restrict__ off_out,
                                                  double inner_tol, double theta) {
    __shared__ double a[kPair * kLdE];
    __shared__ double vt[kPair * kPair];  // transposed rotations: row t is column t of the product
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int k = blockIdx.x;
    const double *g = M + static_cast<int64_t>(kPair) * k * ldm + static_cast<int64_t>(kPair) * k;
    for (int idx = tid; idx < kPair * kPair; idx += 256) {
        const int r = idx >> 6, c = idx & 63;
        a[r * kLdE + c] = r <= c ? g[r * ldm + c] : g[c * ldm + r];
        vt[r * kPair + c] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    double sums[2];
    double off = offdiag(a, red, theta, sums);
    if (tid == 0) {
        off_out[3 * k] = off;
        off_out[3 * k + 1] = sums[0];
        off_out[3 * k + 2] = sums[1];
    }
    for (int sw = 0; sw < kInnerSweeps && off > inner_tol; ++sw) {
        for (int step = 0; step < 63; ++step) {
            double cl = 1.0, sl = 0.0;
            {
                // rotation wave + 4 (lane & 7): rows other waves leave alone in the row pass
                int p, q;
                circle_pair(step, wave + 4 * (lane & 7), &p, &q);
                const double apq = a[p * kLdE + q];
                if (apq != 0.0) {
                    // symmetric Schur rotation zeroing a_pq (smaller root of t^2 + 2 th t - 1 = 0)
                    const double th = (a[q * kLdE + q] - a[p * kLdE + p]) / (2.0 * apq);
                    const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    cl = 1.0 / sqrt(t * t + 1.0);
                    sl = t * cl;
                }
            }
            double cs[8], ss[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                cs[i] = lane_value(cl, i);
                ss[i] = lane_value(sl, i);
            }
            // the 8 rotations touch disjoint rows (columns): all loads of a
            // pass first, then all stores, so their latencies overlap
            int pp[8], qq[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) circle_pair(step, wave + 4 * i, &pp[i], &qq[i]);
            double x[8], y[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {  // rows p, q; lane = column
                x[i] = a[pp[i] * kLdE + lane];
                y[i] = a[qq[i] * kLdE + lane];
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                a[pp[i] * kLdE + lane] = cs[i] * x[i] - ss[i] * y[i];
                a[qq[i] * kLdE + lane] = ss[i] * x[i] + cs[i] * y[i];
            }
            __syncthreads();
            double u[8], v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {  // columns p, q and rotations p, q; lane = row
                x[i] = a[lane * kLdE + pp[i]];
                y[i] = a[lane * kLdE + qq[i]];
                u[i] = vt[pp[i] * kPair + lane];
                v[i] = vt[qq[i] * kPair + lane];
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                a[lane * kLdE + pp[i]] = cs[i] * x[i] - ss[i] * y[i];
                a[lane * kLdE + qq[i]] = ss[i] * x[i] + cs[i] * y[i];
                vt[pp[i] * kPair + lane] = cs[i] * u[i] - ss[i] * v[i];
                vt[qq[i] * kPair + lane] = ss[i] * u[i] + cs[i] * v[i];
            }
            __syncthreads();
        }
        if (sw + 1 < kInnerSweeps) off = offdiag(a, red, theta);
    }
    double *qt = Qt + static_cast<int64_t>(kPair) * k * kPair;
    for (int idx = tid; idx < kPair * kPair; idx += 256) qt[idx] = vt[idx];
}

// Round-0 layout: slot s holds block slot_block[s]: M = P A P^T (zero
// outside n x n), W = the same rows of the identity.
__global__ void k_jac_init(const double *__restrict__ A, int64_t lda, int64_t n, int64_t np,
                           const int *__restrict__ slot_block, double *__restrict__ M, double *__restrict__ W) {
    const int slot = blockIdx.y;
    const int64_t src0 = static_cast<int64_t>(slot_block[slot]) * kBlk;
    for (int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; c < np;
         c += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t sc = static_cast<int64_t>(slot_block[c / kBlk]) * kBlk + c % kBlk;
        for (int r = 0; r < kBlk; ++r) {
            const int64_t src = src0 + r;
            const int64_t dst = (static_cast<int64_t>(slot) * kBlk + r) * np + c;
            M[dst] = (src < n && sc < n) ? A[src * lda + sc] : 0.0;
            W[dst] = src == c ? 1.0 : 0.0;
        }
    }
}

// Step 5: dst = P src P^T (slot s of dst holds slot src_slot[s] of src, rows
// and columns) for blockIdx.z = 0; Wdst = P Wsrc (rows) for blockIdx.z = 1.
__global__ void k_jac_permute(const double *__restrict__ src, double *__restrict__ dst,
                              const double *__restrict__ Wsrc, double *__restrict__ Wdst,
                              const int *__restrict__ src_slot, int64_t np) {
    const int slot = blockIdx.y;
    const bool sym = blockIdx.z == 0;
    const double *from = (sym ? src : Wsrc) + static_cast<int64_t>(src_slot[slot]) * kBlk * np;
    double *to = (sym ? dst : Wdst) + static_cast<int64_t>(slot) * kBlk * np;
    for (int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; c < np;
         c += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t sc = sym ? static_cast<int64_t>(src_slot[c / kBlk]) * kBlk + c % kBlk : c;
        for (int r = 0; r < kBlk; ++r) to[r * np + c] = from[r * np + sc];
    }
}

// lam[c] = M_cc; nrm[c] = |w_c restricted to the first n coordinates|^2
__global__ __launch_bounds__(256) void k_jac_diag(const double *__restrict__ M, const double *__restrict__ W,
                                                  int64_t n, int64_t np, double *__restrict__ lam,
                                                  double *__restrict__ nrm) {
    __shared__ double r2[256];
    const int64_t row = blockIdx.x;
    const double *w = W + row * np;
    double t = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) t = fma(w[i], w[i], t);
    r2[threadIdx.x] = t;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (static_cast<int>(threadIdx.x) < k) r2[threadIdx.x] += r2[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        lam[row] = M[row * np + row];
        nrm[row] = r2[0];
    }
}

// Z[i][j] = scale[j] W[rows[j]][i], i < n, j < nev (through a 32 x 32 LDS tile)
__global__ void k_jac_gather(const double *__restrict__ W, int64_t np, const int *__restrict__ rows,
                             const double *__restrict__ scale, int64_t n, int64_t nev, double *__restrict__ Z,
                             int64_t ldz) {
    __shared__ double tile[32][33];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 32, j0 = static_cast<int64_t>(blockIdx.y) * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
    for (int r = ty; r < 32; r += 8) {
        const int64_t j = j0 + r, i = i0 + tx;
        tile[r][tx] = (j < nev && i < n) ? scale[j] * W[static_cast<int64_t>(rows[j]) * np + i] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = i0 + r, j = j0 + tx;
        if (i < n && j < nev) Z[i * ldz + j] = tile[tx][r];
    }
}

// bad <- 1 if A has a NaN or Inf; part[block] = sum of squares of the block's entries
__global__ __launch_bounds__(256) void k_scan(const double *__restrict__ A, int64_t lda, int64_t n,
                                              int *__restrict__ bad, double *__restrict__ part) {
    __shared__ double r[256];
    int found = 0;
    double ss = 0.0;
    for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < n * n;
         idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double x = A[(idx / n) * lda + idx % n];
        if (!(fabs(x) <= 1.79769313486231570e308)) found = 1;
        else ss = fma(x, x, ss);
    }
    if (found) atomicOr(bad, 1);
    r[threadIdx.x] = ss;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (static_cast<int>(threadIdx.x) < k) r[threadIdx.x] += r[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = r[0];
}

}  // namespace

struct rdm_eig_s {
    ozaki_ctx ctx = nullptr;
    int64_t n = 0, np = 0;
    int S = 0, G = 0, nb = 0, npairs = 0, rounds = 0;
    std::vector<void *> allocs;
    double *X = nullptr, *Y = nullptr;    // M and its ping-pong partner, np x np
    double *W = nullptr, *W2 = nullptr;   // basis rows and their rotation, np x np
    double *Qt = nullptr, *off = nullptr, *lam = nullptr, *nrm = nullptr, *part = nullptr, *scale = nullptr;
    int *slot0 = nullptr, *maps = nullptr, *rows = nullptr, *bad = nullptr;
    int ntiles = 0;
    // native FP64: rows (B = rows of the pair) and columns (B = columns of the pair, transposed)
    TileDesc *tiles = nullptr;
    Term64 *t_rows = nullptr, *t_cols = nullptr;
    OutDesc *outs = nullptr;
    // emulated: Qt slices, pair panels by columns (trans) and by rows
    int32_t *eQ = nullptr, *eR = nullptr, *eC = nullptr;
    int8_t *pQ = nullptr, *pR = nullptr, *pC = nullptr;
    SliceBlock *bR = nullptr, *bC = nullptr;
    SliceTask *eR_t = nullptr, *sR_t = nullptr, *eC_t = nullptr, *sC_t = nullptr;
    int n_eR = 0, n_sR = 0, n_eC = 0, n_sC = 0;
    TermDesc *e_rows = nullptr, *e_cols = nullptr;
    std::vector<double> host_off;
};

namespace {

int ralloc(rdm_eig h, size_t bytes, void **p) {
    hipError_t e = hipMalloc(p, bytes < 256 ? 256 : bytes);
    if (e != hipSuccess) return fail(OZ_ERR_NOMEM, "rdm_eig_create: %zu bytes: %s", bytes, hipGetErrorString(e));
    h->allocs.push_back(*p);
    return OZ_OK;
}

template <typename T>
int rupload(rdm_eig h, const std::vector<T> &v, T **out) {
    void *p;
    int rc = ralloc(h, sizeof(T) * std::max<size_t>(v.size(), 1), &p);
    if (rc) return rc;
    hipError_t e = hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "rdm_eig_create: descriptor upload");
    *out = static_cast<T *>(p);
    return OZ_OK;
}

void rfree(rdm_eig h) {
    for (void *p : h->allocs) hipFree(p);
    delete h;
}

// C rows of each pair <- Q_k^T times the pair's rows of `src` (cols = false)
// or the transpose of its columns (cols = true), in the plan's arithmetic.
int rotate(rdm_eig h, const double *src, double *C, bool cols, hipStream_t s) {
    const int64_t np = h->np;
    hipError_t e;
    if (h->S == 0) {
        Dgemm64Args a{};
        a.tiles = h->tiles;
        a.terms = cols ? h->t_cols : h->t_rows;
        a.outs = h->outs;
        a.ntiles = h->ntiles;
        a.mode = kModeGemm;
        a.tile = 64;
        a.out_base = C;
        a.b_base = src;
        e = launch_dgemm_grouped(cols, a, s);
        return e == hipSuccess ? OZ_OK : hip_fail(e, "rdm_eig: rotation");
    }
    if (cols) {
        if ((e = launch_exponents_grouped(h->bC, h->eC_t, h->n_eC, src, h->eC, h->ctx->d_flags, s)) != hipSuccess ||
            (e = launch_slice_grouped(h->S, h->bC, h->sC_t, h->n_sC, src, h->eC, h->pC, s)) != hipSuccess)
            return hip_fail(e, "rdm_eig: slicing columns");
    } else {
        if ((e = launch_exponents_grouped(h->bR, h->eR_t, h->n_eR, src, h->eR, h->ctx->d_flags, s)) != hipSuccess ||
            (e = launch_slice_grouped(h->S, h->bR, h->sR_t, h->n_sR, src, h->eR, h->pR, s)) != hipSuccess)
            return hip_fail(e, "rdm_eig: slicing rows");
    }
    PairArgs a{};
    a.tiles = h->tiles;
    a.terms = cols ? h->e_cols : h->e_rows;
    a.outs = h->outs;
    a.ntiles = h->ntiles;
    a.mode = kModeGemm;
    a.out_base = C;
    e = launch_pair_grouped(h->S, h->G, 0, a, s);
    (void)np;
    return e == hipSuccess ? OZ_OK : hip_fail(e, "rdm_eig: rotation");
}

// One round (steps 1-5): M in src on entry, in dst on exit.
int enqueue_round(rdm_eig h, int r, const double *src_c, double *dst, double inner_tol, double theta,
                  hipStream_t s) {
    const int64_t np = h->np;
    double *src = const_cast<double *>(src_c);
    hipError_t e;
    hipLaunchKernelGGL(k_pair_eig, dim3(h->npairs), dim3(256), 0, s, src, np, h->Qt,
                       h->off + static_cast<int64_t>(r) * h->npairs * 3, inner_tol, theta);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "rdm_eig: pair eigensolver");
    if (h->S) {
        if ((e = launch_row_exponents(h->Qt, kPair, np, kPair, h->eQ, h->ctx->d_flags, s)) != hipSuccess ||
            (e = launch_slice(h->S, false, h->Qt, kPair, np, kPair, h->eQ, h->pQ, np, s)) != hipSuccess)
            return hip_fail(e, "rdm_eig: slicing Q");
    }
    int rc;
    if ((rc = rotate(h, src, dst, false, s)) != OZ_OK) return rc;    // R = Q^T M
    if ((rc = rotate(h, dst, src, true, s)) != OZ_OK) return rc;     // M' = Q^T R^T
    if ((rc = rotate(h, h->W, h->W2, false, s)) != OZ_OK) return rc;  // W <- Q^T W
    const unsigned cx = static_cast<unsigned>(std::min<int64_t>(ceil_div(np, 256), 16));
    hipLaunchKernelGGL(k_jac_permute, dim3(cx, h->nb, 2), dim3(256), 0, s, src, dst, h->W2, h->W,
                       h->maps + static_cast<int64_t>(r) * h->nb, np);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "rdm_eig: permute");
    return OZ_OK;
}

}  // namespace

extern "C" {

int rdm_eig_create(ozaki_ctx ctx, rdm_eig *out, int64_t n, int slices, int ndiag) {
    if (!out) return fail(OZ_ERR_ARG, "rdm_eig_create: out is NULL");
    *out = nullptr;
    if (!ctx) return fail(OZ_ERR_ARG, "rdm_eig_create: ctx is NULL");
    if (n < 1 || n > kMaxEigN) return fail(OZ_ERR_ARG, "rdm_eig_create: n = %lld (1..%lld)", (long long)n,
                                           (long long)kMaxEigN);
    if (slices != 0 && (slices < 2 || slices > 8)) return fail(OZ_ERR_ARG, "rdm_eig_create: slices = %d", slices);
    const int G = slices ? resolve_ndiag(slices, ndiag) : 0;
    if (slices && !valid_sg(slices, G))
        return fail(OZ_ERR_ARG, "rdm_eig_create: ndiag = %d for slices = %d (use S, S+1 or 2S-1)", ndiag, slices);
    const int64_t np = round_up(n, kPair);
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    rdm_eig h = new rdm_eig_s();
    h->ctx = ctx;
    h->n = n;
    h->np = np;
    h->S = slices;
    h->G = G;
    h->nb = static_cast<int>(np / kBlk);
    h->npairs = h->nb / 2;
    h->rounds = h->nb - 1;
    int rc;
    void *p;
    const size_t mat = sizeof(double) * static_cast<size_t>(np) * np;
#define OZ_RA(field, bytes) \
    if ((rc = ralloc(h, (bytes), &p)) != OZ_OK) { rfree(h); return rc; } \
    h->field = static_cast<decltype(h->field)>(p);
    OZ_RA(X, mat)
    OZ_RA(Y, mat)
    OZ_RA(W, mat)
    OZ_RA(W2, mat)
    OZ_RA(Qt, sizeof(double) * np * kPair)
    OZ_RA(off, sizeof(double) * h->rounds * h->npairs * 3)
    OZ_RA(lam, sizeof(double) * np)
    OZ_RA(nrm, sizeof(double) * np)
    OZ_RA(scale, sizeof(double) * np)
    OZ_RA(rows, sizeof(int) * np)
    OZ_RA(bad, sizeof(int) * 4)
    OZ_RA(part, sizeof(double) * kScanBlocks)
#undef OZ_RA
    // circle schedule over the nb blocks
    std::vector<int> a(h->nb);
    std::iota(a.begin(), a.end(), 0);
    std::vector<std::vector<int>> slot_block(h->rounds, std::vector<int>(h->nb));
    for (int r = 0; r < h->rounds; ++r) {
        for (int k = 0; k < h->npairs; ++k) {
            slot_block[r][2 * k] = a[k];
            slot_block[r][2 * k + 1] = a[h->nb - 1 - k];
        }
        std::rotate(a.begin() + 1, a.end() - 1, a.end());
    }
    std::vector<int> maps(static_cast<size_t>(h->rounds) * h->nb);
    for (int r = 0; r < h->rounds; ++r) {
        const std::vector<int> &cur = slot_block[r], &nxt = slot_block[(r + 1) % h->rounds];
        std::vector<int> slot_of(h->nb);
        for (int sl = 0; sl < h->nb; ++sl) slot_of[cur[sl]] = sl;
        for (int sl = 0; sl < h->nb; ++sl) maps[static_cast<size_t>(r) * h->nb + sl] = slot_of[nxt[sl]];
    }
    if ((rc = rupload(h, slot_block[0], &h->slot0)) || (rc = rupload(h, maps, &h->maps))) {
        rfree(h);
        return rc;
    }
    // tiles: pair k x 64-column tile c, row offset 64k into Qt and the output
    const int ctiles = static_cast<int>(np / 64);
    std::vector<TileDesc> tiles;
    for (int k = 0; k < h->npairs; ++k)
        for (int c = 0; c < ctiles; ++c) tiles.push_back(TileDesc{k, k + 1, kPair * k, 64 * c, 0, 0});
    h->ntiles = static_cast<int>(tiles.size());
    // outputs and B operands are element offsets from the buffers passed at launch
    const std::vector<OutDesc> outs{OutDesc{nullptr, np, static_cast<int32_t>(np), static_cast<int32_t>(np)}};
    if ((rc = rupload(h, tiles, &h->tiles)) || (rc = rupload(h, outs, &h->outs))) {
        rfree(h);
        return rc;
    }
    if (slices == 0) {
        std::vector<Term64> tr, tc;
        for (int k = 0; k < h->npairs; ++k) {
            const intptr_t ro = static_cast<intptr_t>(kPair) * k * np, co = static_cast<intptr_t>(kPair) * k;
            tr.push_back(Term64{h->Qt, reinterpret_cast<const double *>(ro), kPair, np, kPair, 0, 1.0});
            tc.push_back(Term64{h->Qt, reinterpret_cast<const double *>(co), kPair, np, kPair, 0, 1.0});
        }
        if ((rc = rupload(h, tr, &h->t_rows)) || (rc = rupload(h, tc, &h->t_cols))) {
            rfree(h);
            return rc;
        }
    } else {
        if ((rc = ralloc(h, sizeof(int32_t) * np, &p)) != OZ_OK) { rfree(h); return rc; }
        h->eQ = static_cast<int32_t *>(p);
        if ((rc = ralloc(h, static_cast<size_t>(slices) * np * kPair, &p)) != OZ_OK) { rfree(h); return rc; }
        h->pQ = static_cast<int8_t *>(p);
        // B operands: the pair's 64 rows grouped by columns (R = Q^T M, W), or
        // the pair's 64 columns grouped by rows (Q^T R^T)
        SliceSet setR, setC;
        std::vector<int64_t> eoR, poR, eoC, poC;
        for (int k = 0; k < h->npairs; ++k) {
            int64_t eo, po;
            setR.add(static_cast<int64_t>(kPair) * k * np, np, np, kPair, true, slices, &eo, &po);
            eoR.push_back(eo);
            poR.push_back(po);
            setC.add(static_cast<int64_t>(kPair) * k, np, np, kPair, false, slices, &eo, &po);
            eoC.push_back(eo);
            poC.push_back(po);
        }
        if ((rc = rupload(h, setR.blocks, &h->bR)) || (rc = rupload(h, setR.etasks, &h->eR_t)) ||
            (rc = rupload(h, setR.stasks, &h->sR_t)) || (rc = rupload(h, setC.blocks, &h->bC)) ||
            (rc = rupload(h, setC.etasks, &h->eC_t)) || (rc = rupload(h, setC.stasks, &h->sC_t))) {
            rfree(h);
            return rc;
        }
        h->n_eR = static_cast<int>(setR.etasks.size());
        h->n_sR = static_cast<int>(setR.stasks.size());
        h->n_eC = static_cast<int>(setC.etasks.size());
        h->n_sC = static_cast<int>(setC.stasks.size());
        if ((rc = ralloc(h, sizeof(int32_t) * setR.e_total, &p)) != OZ_OK) { rfree(h); return rc; }
        h->eR = static_cast<int32_t *>(p);
        if ((rc = ralloc(h, setR.p_total, &p)) != OZ_OK) { rfree(h); return rc; }
        h->pR = static_cast<int8_t *>(p);
        if ((rc = ralloc(h, sizeof(int32_t) * setC.e_total, &p)) != OZ_OK) { rfree(h); return rc; }
        h->eC = static_cast<int32_t *>(p);
        if ((rc = ralloc(h, setC.p_total, &p)) != OZ_OK) { rfree(h); return rc; }
        h->pC = static_cast<int8_t *>(p);
        std::vector<TermDesc> tr, tc;
        for (int k = 0; k < h->npairs; ++k) {
            tr.push_back(TermDesc{h->pQ, h->eQ, h->pR + poR[k], h->eR + eoR[k], np, np, kPair / kKB, 0, 1.0});
            tc.push_back(TermDesc{h->pQ, h->eQ, h->pC + poC[k], h->eC + eoC[k], np, np, kPair / kKB, 0, 1.0});
        }
        if ((rc = rupload(h, tr, &h->e_rows)) || (rc = rupload(h, tc, &h->e_cols))) {
            rfree(h);
            return rc;
        }
    }
    *out = h;
    return OZ_OK;
}

int rdm_eig_solve(rdm_eig h, const double *A, int64_t lda, int64_t nev, double *evals, double *Z, int64_t ldz,
                  double tol, int max_sweeps, rdm_eig_info *info, void *stream) {
    if (!h) return fail(OZ_ERR_ARG, "rdm_eig_solve: NULL solver");
    const int64_t n = h->n, np = h->np;
    if (!A || lda < n) return fail(OZ_ERR_ARG, "rdm_eig_solve: A is NULL or lda < n");
    if (nev < 0 || nev > n) return fail(OZ_ERR_ARG, "rdm_eig_solve: nev = %lld (0..%lld)", (long long)nev,
                                        (long long)n);
    if (nev > 0 && (!evals || !Z || ldz < nev)) return fail(OZ_ERR_ARG, "rdm_eig_solve: evals / Z / ldz");
    if (max_sweeps < 1) return fail(OZ_ERR_ARG, "rdm_eig_solve: max_sweeps = %d", max_sweeps);
    if (!(tol >= 0.0)) return fail(OZ_ERR_ARG, "rdm_eig_solve: tol");
    // unit roundoff of the arithmetic in use: FP64, or the emulation's 8S - 1 bits
    const double u_eff = h->S ? std::max(0x1p-53, std::ldexp(1.0, 1 - 8 * h->S)) : 0x1p-53;
    if (tol == 0.0) tol = 4.0 * std::sqrt(static_cast<double>(np)) * u_eff;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = hipSetDevice(h->ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    int hb[1] = {0};
    if ((e = hipMemcpyAsync(h->bad, hb, sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "rdm_eig_solve: flag");
    const unsigned scan_blocks = static_cast<unsigned>(std::min<int64_t>(ceil_div(n * n, 256), kScanBlocks));
    hipLaunchKernelGGL(k_scan, dim3(scan_blocks), dim3(256), 0, s, A, lda, n, h->bad, h->part);
    std::vector<double> part(scan_blocks);
    if ((e = hipMemcpyAsync(hb, h->bad, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(part.data(), h->part, sizeof(double) * scan_blocks, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "rdm_eig_solve: finiteness check");
    if (hb[0]) return fail(OZ_ERR_ARG, "rdm_eig_solve: A has NaN or Inf entries");
    double fro2 = 0.0;
    for (double x : part) fro2 += x;
    const double fro = std::sqrt(fro2);
    const double abs_tol = tol * fro;
    hipLaunchKernelGGL(k_jac_init, dim3(static_cast<unsigned>(std::min<int64_t>(ceil_div(np, 256), 16)), h->nb),
                       dim3(256), 0, s, A, lda, n, np, h->slot0, h->X, h->W);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "rdm_eig_solve: init");
    int status = OZ_MAX_ITER, sweeps = 0, no_progress = 0;
    double best = INFINITY, last = INFINITY;
    double *cur = h->X, *other = h->Y;
    h->host_off.resize(static_cast<size_t>(h->rounds) * h->npairs * 3);
    std::vector<double> lam(np), nrm(np);
    // Diagonal of M over the squared basis norms (Rayleigh quotients) and
    // the basis rows inside the first n coordinates (the others are padding).
    auto diagonal = [&](std::vector<int> *rows) -> int {
        hipLaunchKernelGGL(k_jac_diag, dim3(static_cast<unsigned>(np)), dim3(256), 0, s, cur, h->W, n, np, h->lam,
                           h->nrm);
        if ((e = hipMemcpyAsync(lam.data(), h->lam, sizeof(double) * np, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(nrm.data(), h->nrm, sizeof(double) * np, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(e, "rdm_eig_solve: eigenvalues");
        rows->clear();
        for (int64_t c = 0; c < np; ++c)
            if (nrm[c] > 0.5) rows->push_back(static_cast<int>(c));
        if (static_cast<int64_t>(rows->size()) != n)
            return fail(OZ_ERR_HIP, "rdm_eig_solve: %zu basis rows inside the first %lld coordinates (expected %lld)",
                        rows->size(), (long long)n, (long long)n);
        // the emulated rotations are orthogonal only to the emulation's precision
        for (int c : *rows) lam[c] /= nrm[c];
        std::stable_sort(rows->begin(), rows->end(), [&](int x, int y) { return lam[x] > lam[y]; });
        return OZ_OK;
    };
    std::vector<int> rows;
    // Rows whose diagonal is below theta are outside the wanted part: their
    // mutual couplings are exempt from tol (nev = n: none is).  theta is the
    // midpoint of the gap at the nev-th value of the previous sweep.
    double theta = -INFINITY;
    for (int sw = 0; sw < max_sweeps && fro > 0.0; ++sw) {
        for (int r = 0; r < h->rounds; ++r) {
            const int rc = enqueue_round(h, r, cur, other, 0.1 * abs_tol, theta, s);
            if (rc != OZ_OK) return rc;
            std::swap(cur, other);
        }
        sweeps = sw + 1;
        if ((e = hipMemcpyAsync(h->host_off.data(), h->off, sizeof(double) * h->host_off.size(),
                                hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "rdm_eig_solve: sweep");
        int rc = diagonal(&rows);
        if (rc != OZ_OK) return rc;
        double sum = 0.0, exempt = 0.0;
        last = 0.0;
        for (size_t i = 0; i < h->host_off.size(); i += 3) {
            last = std::max(last, h->host_off[i]);
            sum += h->host_off[i + 1];
            exempt += h->host_off[i + 2];
        }
        last /= fro;
        // the wanted rows are decoupled to tol, and by Weyl's bound the
        // exempt couplings cannot lift an unwanted eigenvalue above them
        bool separated = true;
        if (nev < n) {
            const double lo = lam[rows[nev - 1 < 0 ? 0 : nev - 1]], hi = lam[rows[nev]];
            separated = nev == 0 || (hi < theta && theta <= lo && hi + std::sqrt(exempt) < lo);
            theta = nev == 0 ? INFINITY : 0.5 * (lo + hi);
        }
        if (last <= tol && separated) {
            status = OZ_CONVERGED;
            break;
        }
        // three sweeps in a row without halving the best off-diagonal mass: the arithmetic's floor
        no_progress = sum > 0.5 * best ? no_progress + 1 : 0;
        best = std::min(best, sum);
        if (no_progress >= 3) {
            status = OZ_STAGNATED;
            break;
        }
    }
    if (fro == 0.0) {
        status = OZ_CONVERGED;
        last = 0.0;
    }
    {
        const int rc = diagonal(&rows);
        if (rc != OZ_OK) return rc;
    }
    double trace = 0.0;
    for (int c : rows) trace += lam[c];
    if (nev > 0) {
        std::vector<double> ev(nev), scale(nev);
        for (int64_t j = 0; j < nev; ++j) {
            ev[j] = lam[rows[j]];
            scale[j] = 1.0 / std::sqrt(nrm[rows[j]]);
        }
        if ((e = hipMemcpyAsync(h->rows, rows.data(), sizeof(int) * nev, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(h->scale, scale.data(), sizeof(double) * nev, hipMemcpyHostToDevice, s)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(evals, ev.data(), sizeof(double) * nev, hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_fail(e, "rdm_eig_solve: output");
        hipLaunchKernelGGL(k_jac_gather, dim3(static_cast<unsigned>(ceil_div(n, 32)), static_cast<unsigned>(ceil_div(nev, 32))),
                           dim3(256), 0, s, h->W, np, h->rows, h->scale, n, nev, Z, ldz);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "rdm_eig_solve: gather");
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "rdm_eig_solve: gather");
    }
    if (info) *info = rdm_eig_info{sweeps, status, last, trace};
    return OZ_OK;
}

int rdm_eig_destroy(rdm_eig h) {
    if (!h) return OZ_OK;
    hipSetDevice(h->ctx->device);
    hipDeviceSynchronize();
    rfree(h);
    return OZ_OK;
}

size_t ozaki_renormalize_workspace_bytes(int64_t n, int64_t D, int slices, int ndiag) {
    if (n < 0 || D < 0) return 0;
    size_t t = align256(sizeof(double) * static_cast<size_t>(n) * D);
    if (slices == 0) return t;
    const size_t w1 = ozaki_dgemm_workspace_bytes(n, D, n, slices, ndiag);
    const size_t w2 = ozaki_dgemm_workspace_bytes(D, D, n, slices, ndiag);
    return t + std::max(w1, w2);
}

int ozaki_renormalize(ozaki_ctx ctx, int64_t n, int64_t D, const double *U, int64_t ldu, int count,
                      const double *const *ops, int64_t ldo, double *const *outs, int64_t ldout, int slices,
                      int ndiag, void *workspace, size_t workspace_bytes, void *stream) {
    if (!ctx) return fail(OZ_ERR_ARG, "ozaki_renormalize: ctx is NULL");
    if (n < 0 || D < 0 || D > n || count < 0) return fail(OZ_ERR_ARG, "ozaki_renormalize: sizes");
    if (count > 0 && (!ops || !outs)) return fail(OZ_ERR_ARG, "ozaki_renormalize: ops / outs is NULL");
    if (ldu < (D > 1 ? D : 1) || ldo < (n > 1 ? n : 1) || ldout < (D > 1 ? D : 1))
        return fail(OZ_ERR_ARG, "ozaki_renormalize: leading dimension");
    if (n == 0 || D == 0 || count == 0) return OZ_OK;
    const size_t need = ozaki_renormalize_workspace_bytes(n, D, slices, ndiag);
    if (!workspace || workspace_bytes < need)
        return fail(OZ_ERR_WORKSPACE, "ozaki_renormalize: workspace %zu bytes, need %zu", workspace_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(OZ_ERR_WORKSPACE, "ozaki_renormalize: workspace not 256-byte aligned");
    double *T = static_cast<double *>(workspace);
    const size_t tb = align256(sizeof(double) * static_cast<size_t>(n) * D);
    void *gw = slices ? static_cast<char *>(workspace) + tb : nullptr;
    const size_t gwb = slices ? workspace_bytes - tb : 0;
    for (int k = 0; k < count; ++k) {
        if (!ops[k] || !outs[k]) return fail(OZ_ERR_ARG, "ozaki_renormalize: operator %d is NULL", k);
        // T = O_k U (n x D), then O'_k = U^T T (D x D)
        int rc = ozaki_dgemm(ctx, 'N', 'N', n, D, n, 1.0, ops[k], ldo, U, ldu, 0.0, T, D, slices, ndiag, gw, gwb,
                             stream);
        if (rc != OZ_OK) return rc;
        rc = ozaki_dgemm(ctx, 'T', 'N', D, D, n, 1.0, U, ldu, T, D, 0.0, outs[k], ldout, slices, ndiag, gw, gwb,
                         stream);
        if (rc != OZ_OK) return rc;
    }
    return OZ_OK;
}

}  // extern "C"
