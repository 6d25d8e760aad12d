// Davidson iteration for the lowest eigenpair of H_eff (the Krylov solver of
// the second DMRG subroutine, "Theory of TNS/DMRG"; stopped on the residual
// norm as in "Numerical procedure").  The matvec is heff_apply (emulated or
// native); everything else runs in FP64 on the device:
//
//   Rayleigh-Ritz   one-workgroup cyclic Jacobi (round-robin ordering, all
//                   disjoint rotations of a round applied together) on the
//                   m x m projected matrix, m <= 64;
//   Ritz vector     x = V^T y, Hx = W^T y, r = Hx - theta x, rho = |r|;
//   correction      t = r / (diag(H) - theta), |den| >= 1e-8;
//   orthogonalise   classical Gram-Schmidt twice against V, fall back to r
//                   when |t| < 1e-10, normalise;
//   expand          W[m] = H V[m] and the new column of V^T W.
//
// All reductions use a fixed partition and a fixed tree, so a run is
// bit-reproducible.  The host reads (theta, rho) once per step.
#include <cmath>
#include <type_traits>
#include <vector>

#include "runtime.h"

using namespace oz;

namespace {

constexpr int kDotThreads = 256;

int dot_blocks(int64_t n) {
    const int64_t b = ceil_div(n, kDotThreads * 4);
    return static_cast<int>(b < 1 ? 1 : (b > 512 ? 512 : b));
}

__device__ inline double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Rows of a launch counted on the device: with m non-null the rows are
// *m + add (the grid covers the largest count, the rows past it return),
// else the grid's.  The Davidson basis size lives on the device, so one
// captured step serves every basis size.
struct DevRows {
    const int *m;
    int add;
    __device__ bool skip(int row) const { return m && row >= *m + add; }
};

// partial[row][blk] = sum over this block's share of A[row][i] * v[i]
__global__ __launch_bounds__(kDotThreads) void k_dots_partial(const double *__restrict__ A, int64_t lda, const double *__restrict__ v,
                                                              int64_t n, double *__restrict__ partial, const int *gate,
                                                              DevRows rows) {
    if (gate && *gate == 0) return;
    if (rows.skip(blockIdx.y)) return;
    __shared__ double sh[kDotThreads];
    const int row = blockIdx.y;
    const double *a = A + row * lda;
    double acc = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        acc = fma(a[i], v[i], acc);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[static_cast<int64_t>(row) * gridDim.x + blockIdx.x] = s;
}

// out[row * out_stride] = sum of the row's partials; optional mirror out2.
// With rows.m set, out and out2 move by *rows.m times out_mscale / out2_mscale.
__global__ __launch_bounds__(kDotThreads) void k_dots_final(const double *__restrict__ partial, int nblk, double *out, int64_t out_stride,
                                                            double *out2, int64_t out2_stride, const int *gate,
                                                            DevRows rows, int64_t out_mscale, int64_t out2_mscale) {
    if (gate && *gate == 0) return;
    if (rows.skip(blockIdx.x)) return;
    __shared__ double sh[kDotThreads];
    const int row = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += partial[static_cast<int64_t>(row) * nblk + b];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        const int64_t m = rows.m ? *rows.m : 0;
        out[m * out_mscale + row * out_stride] = s;
        if (out2) out2[m * out2_mscale + row * out2_stride] = s;
    }
}

// Lowest eigenpair of the symmetric m x m matrix G (leading dimension ldg) by
// cyclic Jacobi with the round-robin pairing; writes theta and y (largest
// |y_i| made positive).  One workgroup of 256 threads, m <= 64.
__global__ __launch_bounds__(256) void k_jacobi(const double *__restrict__ G, int ldg, int m_arg, const int *m_dev,
                                                double *__restrict__ y, double *__restrict__ theta_out) {
    const int m = m_dev ? *m_dev : m_arg;
    __shared__ double A[64][65];
    __shared__ double Vv[64][65];
    __shared__ double cs[32], sn[32];
    __shared__ int pp[32], qq[32];
    __shared__ double red[256];
    __shared__ int done;
    const int t = threadIdx.x;
    for (int i = t; i < m * m; i += blockDim.x) {
        const int r = i / m, c = i % m;
        A[r][c] = G[r * ldg + c];
        Vv[r][c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int me = (m + 1) & ~1;  // even number of players (one dummy when m is odd)
    for (int sweep = 0; sweep < 30 && m > 1; ++sweep) {
        // convergence test: off(A) <= 1e-14 ||A||_F
        double off = 0.0, tot = 0.0;
        for (int i = t; i < m * m; i += blockDim.x) {
            const int r = i / m, c = i % m;
            const double v = A[r][c] * A[r][c];
            tot += v;
            if (r != c) off += v;
        }
        const double soff = block_sum(off, red);
        const double stot = block_sum(tot, red);
        if (t == 0) done = (sqrt(soff) <= 1e-14 * sqrt(stot)) ? 1 : 0;
        __syncthreads();
        if (done) break;
        for (int round = 0; round < me - 1; ++round) {
            // round-robin: player me-1 fixed, the others rotate
            if (t < me / 2) {
                int a, b;
                if (t == 0) {
                    a = me - 1;
                    b = round;
                } else {
                    a = (round + t) % (me - 1);
                    b = (round - t + (me - 1)) % (me - 1);
                }
                const int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double apq = A[p][q];
                    if (apq != 0.0) {
                        const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
                        const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(tt * tt + 1.0);
                        s = tt * c;
                    }
                }
                cs[t] = c;
                sn[t] = s;
                pp[t] = p;
                qq[t] = q < m ? q : -1;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int i = t; i < (me / 2) * m; i += blockDim.x) {
                const int k = i / m, c = i % m;
                if (qq[k] < 0) continue;
                const int p = pp[k], q = qq[k];
                const double ap = A[p][c], aq = A[q][c];
                A[p][c] = cs[k] * ap - sn[k] * aq;
                A[q][c] = sn[k] * ap + cs[k] * aq;
            }
            __syncthreads();
            // columns: A <- A J, eigenvectors V <- V J
            for (int i = t; i < (me / 2) * m; i += blockDim.x) {
                const int k = i / m, r = i % m;
                if (qq[k] < 0) continue;
                const int p = pp[k], q = qq[k];
                const double ap = A[r][p], aq = A[r][q];
                A[r][p] = cs[k] * ap - sn[k] * aq;
                A[r][q] = sn[k] * ap + cs[k] * aq;
                const double vp = Vv[r][p], vq = Vv[r][q];
                Vv[r][p] = cs[k] * vp - sn[k] * vq;
                Vv[r][q] = sn[k] * vp + cs[k] * vq;
            }
            __syncthreads();
        }
    }
    if (t == 0) {
        int best = 0;
        for (int i = 1; i < m; ++i)
            if (A[i][i] < A[best][best]) best = i;
        int big = 0;
        for (int i = 1; i < m; ++i)
            if (fabs(Vv[i][best]) > fabs(Vv[big][best])) big = i;
        const double sgn = Vv[big][best] < 0 ? -1.0 : 1.0;
        for (int i = 0; i < m; ++i) y[i] = sgn * Vv[i][best];
        *theta_out = A[best][best];
    }
}

// x = V^T y, hx = W^T y, r = hx - theta x, partial sums of r^2.
__global__ __launch_bounds__(kDotThreads) void k_ritz(const double *__restrict__ V, const double *__restrict__ W, int64_t n,
                                                      const int *m_dev, const double *__restrict__ y, const double *__restrict__ theta,
                                                      double *__restrict__ x, double *__restrict__ hx, double *__restrict__ r,
                                                      double *__restrict__ partial) {
    const int m = *m_dev;
    __shared__ double sh[kDotThreads];
    const double th = *theta;
    double acc = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double xi = 0.0, hi = 0.0;
        for (int j = 0; j < m; ++j) {
            xi = fma(y[j], V[j * n + i], xi);
            hi = fma(y[j], W[j * n + i], hi);
        }
        const double ri = hi - th * xi;
        x[i] = xi;
        hx[i] = hi;
        r[i] = ri;
        acc = fma(ri, ri, acc);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_precond(const double *__restrict__ r, const double *__restrict__ hdiag,
                          const double *__restrict__ theta, double *__restrict__ t, int64_t n) {
    const double th = *theta;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double den = hdiag[i] - th;
        if (fabs(den) < 1e-8) den = copysign(1e-8, den);
        t[i] = r[i] / den;
    }
}

// t -= V^T c  (c: m projection coefficients)
__global__ void k_project(const double *__restrict__ V, int64_t n, int m_arg, const int *m_dev,
                          const double *__restrict__ c, double *__restrict__ t, const int *gate) {
    if (gate && *gate == 0) return;
    const int m = m_dev ? *m_dev : m_arg;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s = fma(c[j], V[j * n + i], s);
        t[i] = t[i] - s;
    }
}

// when |t|^2 < 1e-20 replace t by r and raise the gate for a second pass
__global__ void k_fallback(const double *__restrict__ nrm2, const double *__restrict__ r, double *__restrict__ t,
                           int64_t n, int *gate) {
    const bool fb = *nrm2 < 1e-20;
    if (blockIdx.x == 0 && threadIdx.x == 0) *gate = fb ? 1 : 0;
    if (!fb) return;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        t[i] = r[i];
}

// out (moved by *m_dev rows of n when m_dev is set) = t / sqrt(nrm2); the
// same values into out2 when it is set
__global__ void k_scale_into(const double *__restrict__ t, const double *__restrict__ nrm2, double *__restrict__ out,
                             int64_t n, const int *m_dev = nullptr, double *__restrict__ out2 = nullptr) {
    const double inv = 1.0 / sqrt(*nrm2);
    double *o = out + (m_dev ? static_cast<int64_t>(*m_dev) * n : 0);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double v = t[i] * inv;
        o[i] = v;
        if (out2) out2[i] = v;
    }
}

// collapse the basis to the Ritz pair when it is full (*m_dev == mmax):
// G = [theta], zero elsewhere, and the basis size becomes 1
__global__ void k_collapse_g(double *G, int ldg, int mmax, const double *theta, int *m_dev) {
    if (*m_dev != mmax) return;
    for (int i = threadIdx.x; i < mmax * mmax; i += blockDim.x) G[(i / mmax) * ldg + i % mmax] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        G[0] = *theta;
        *m_dev = 1;
    }
}

// dst (moved by *m_dev rows of n) = src; with full set, only when the basis
// is full (*m_dev == full), into row 0 (the collapse to the Ritz pair)
__global__ void k_copy_row(const double *__restrict__ src, double *__restrict__ dst, int64_t n, const int *m_dev,
                           int full) {
    const int m = *m_dev;
    if (full && m != full) return;
    double *d = dst + (full ? 0 : static_cast<int64_t>(m) * n);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        d[i] = src[i];
}

// *m_dev += 1 (the basis gained a vector)
__global__ void k_bump(int *m_dev) {
    if (threadIdx.x == 0) *m_dev += 1;
}

// (theta, rho^2) into the pinned host buffer the step reads after its sync
__global__ void k_publish(const double *__restrict__ scal, double *host) {
    if (threadIdx.x < 2) host[threadIdx.x] = scal[threadIdx.x];
}

unsigned grid_n(int64_t n) {
    const int64_t g = ceil_div(n, 256);
    return static_cast<unsigned>(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

struct davidson_s {
    ozaki_ctx ctx = nullptr;
    heff_plan H = nullptr;
    int64_t n = 0;
    int m_max = 0, max_iter = 0;
    double tol = 0;
    std::vector<void *> allocs;
    double *V = nullptr, *W = nullptr, *G = nullptr, *hdiag = nullptr;
    // Ritz vectors of two consecutive Rayleigh-Ritz solves: xs[cur] is the
    // latest, xs[rep] the one whose theta the last step reported
    double *xs[2] = {nullptr, nullptr};
    int cur = 0, rep = 0;
    double *hx = nullptr, *r = nullptr, *t = nullptr;
    double *mv_in = nullptr, *mv_out = nullptr;  // the matvec's fixed input and output
    double *y = nullptr, *coef = nullptr, *partial = nullptr, *scal = nullptr;  // scal: theta, rho2, nrm2
    int *gate = nullptr;
    int *m_dev = nullptr;  // the basis size on the device (the host keeps m too)
    double *host = nullptr;  // pinned: theta, rho2 of the latest Rayleigh-Ritz solve
    int m = 0, iter = 0, status = OZ_OK;
    std::vector<double> hist;
    // Replay: the launches that follow a step's decision (correction, basis
    // update, matvec, next Rayleigh-Ritz) read the basis size from the
    // device and use fixed matvec buffers, so they depend only on which Ritz
    // buffer is current: two graphs serve every step.
    bool use_graphs = true;
    hipStream_t cap = nullptr;
    hipGraphExec_t graphs[2] = {nullptr, nullptr};  // per current Ritz buffer
};

namespace {

int dalloc(davidson d, size_t bytes, void **p) {
    hipError_t e = hipMalloc(p, bytes < 8 ? 8 : bytes);
    if (e != hipSuccess) return fail(OZ_ERR_NOMEM, "davidson_create: %zu bytes: %s", bytes, hipGetErrorString(e));
    d->allocs.push_back(*p);
    return OZ_OK;
}

void dfree(davidson d) {
    for (auto g : d->graphs)
        if (g) hipGraphExecDestroy(g);
    if (d->cap) hipStreamDestroy(d->cap);
    for (void *p : d->allocs) hipFree(p);
    if (d->host) hipHostFree(d->host);
    delete d;
}

// out[i] = row_i(A) . v for i < rows (rows with stride lda), into out[i * out_stride]
hipError_t dots(davidson d, const double *A, int64_t lda, int rows, const double *v, double *out,
                int64_t out_stride, double *out2, int64_t out2_stride, const int *gate, hipStream_t s) {
    const int nb = dot_blocks(d->n);
    hipLaunchKernelGGL(k_dots_partial, dim3(nb, rows), dim3(kDotThreads), 0, s, A, lda, v, d->n, d->partial, gate,
                       DevRows{nullptr, 0});
    hipLaunchKernelGGL(k_dots_final, dim3(rows), dim3(kDotThreads), 0, s, d->partial, nb, out, out_stride, out2,
                       out2_stride, gate, DevRows{nullptr, 0}, 0, 0);
    return hipGetLastError();
}

// The same over *m_dev + add rows of A (the grid covers m_max + 1); out and
// out2 move by *m_dev times out_mscale / out2_mscale.
hipError_t dots_m(davidson d, const double *A, int64_t lda, int add, const double *v, double *out,
                  int64_t out_stride, int64_t out_mscale, double *out2, int64_t out2_stride, int64_t out2_mscale,
                  const int *gate, hipStream_t s) {
    const int nb = dot_blocks(d->n);
    const int rows = d->m_max + add;
    hipLaunchKernelGGL(k_dots_partial, dim3(nb, rows), dim3(kDotThreads), 0, s, A, lda, v, d->n, d->partial, gate,
                       DevRows{d->m_dev, add});
    hipLaunchKernelGGL(k_dots_final, dim3(rows), dim3(kDotThreads), 0, s, d->partial, nb, out, out_stride, out2,
                       out2_stride, gate, DevRows{d->m_dev, add}, out_mscale, out2_mscale);
    return hipGetLastError();
}

// V[m] := normalised, orthogonalised t; W[m] = H V[m]; new column of G;
// m += 1.  m is the device's basis size.
int expand(davidson d, hipStream_t s) {
    hipError_t e;
    const int64_t n = d->n;
    double *nrm2 = d->scal + 2;
    for (int pass = 0; pass < 2; ++pass) {
        if ((e = dots_m(d, d->V, n, 0, d->t, d->coef, 1, 0, nullptr, 0, 0, nullptr, s)) != hipSuccess)
            return hip_fail(e, "davidson: projection");
        hipLaunchKernelGGL(k_project, dim3(grid_n(n)), dim3(256), 0, s, d->V, n, 0, d->m_dev, d->coef, d->t, nullptr);
    }
    if ((e = dots(d, d->t, n, 1, d->t, nrm2, 1, nullptr, 0, nullptr, s)) != hipSuccess) return hip_fail(e, "davidson: norm");
    hipLaunchKernelGGL(k_fallback, dim3(grid_n(n)), dim3(256), 0, s, nrm2, d->r, d->t, n, d->gate);
    for (int pass = 0; pass < 2; ++pass) {
        dots_m(d, d->V, n, 0, d->t, d->coef, 1, 0, nullptr, 0, 0, d->gate, s);
        hipLaunchKernelGGL(k_project, dim3(grid_n(n)), dim3(256), 0, s, d->V, n, 0, d->m_dev, d->coef, d->t, d->gate);
    }
    dots(d, d->t, n, 1, d->t, nrm2, 1, nullptr, 0, d->gate, s);
    // V[m] and the matvec's input get the same values
    hipLaunchKernelGGL(k_scale_into, dim3(grid_n(n)), dim3(256), 0, s, d->t, nrm2, d->V, n, d->m_dev, d->mv_in);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "davidson: orthogonalisation");
    int rc = heff_apply(d->H, d->mv_in, d->mv_out, s);
    if (rc != OZ_OK) return rc;
    hipLaunchKernelGGL(k_copy_row, dim3(grid_n(n)), dim3(256), 0, s, d->mv_out, d->W, n, d->m_dev, 0);
    // G[i][m] = G[m][i] = V[i] . W[m], i <= m
    if ((e = dots_m(d, d->V, n, 1, d->mv_out, d->G, d->m_max, 1, d->G, 1, d->m_max, nullptr, s)) != hipSuccess)
        return hip_fail(e, "davidson: projected column");
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, s, d->m_dev);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "davidson: basis size");
    return OZ_OK;
}

// Rayleigh-Ritz on the device's basis of m vectors, the Ritz pair into x_out
// (and hx, r), rho^2, and (theta, rho^2) published to the pinned host buffer.
int rayleigh_ritz(davidson d, double *x_out, hipStream_t s) {
    const int64_t n = d->n;
    double *theta = d->scal, *rho2 = d->scal + 1;
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(256), 0, s, d->G, d->m_max, 0, d->m_dev, d->y, theta);
    const int nb = dot_blocks(n);
    hipLaunchKernelGGL(k_ritz, dim3(nb), dim3(kDotThreads), 0, s, d->V, d->W, n, d->m_dev, d->y, theta, x_out, d->hx,
                       d->r, d->partial);
    hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(kDotThreads), 0, s, d->partial, nb, rho2, 1, nullptr, 0, nullptr,
                       DevRows{nullptr, 0}, 0, 0);
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, d->scal, d->host);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? OZ_OK : hip_fail(e, "davidson: Rayleigh-Ritz");
}

// Everything a continuing step does after its decision, with current Ritz
// buffer c: correction, collapse when the basis is full, orthogonalisation
// and matvec, then the next Rayleigh-Ritz into xs[c ^ 1].
int step_tail(davidson d, int c, hipStream_t s) {
    const int64_t n = d->n;
    const double *theta = d->scal;
    hipLaunchKernelGGL(k_precond, dim3(grid_n(n)), dim3(256), 0, s, d->r, d->hdiag, theta, d->t, n);
    hipLaunchKernelGGL(k_copy_row, dim3(grid_n(n)), dim3(256), 0, s, d->xs[c], d->V, n, d->m_dev, d->m_max);
    hipLaunchKernelGGL(k_copy_row, dim3(grid_n(n)), dim3(256), 0, s, d->hx, d->W, n, d->m_dev, d->m_max);
    hipLaunchKernelGGL(k_collapse_g, dim3(1), dim3(256), 0, s, d->G, d->m_max, d->m_max, theta, d->m_dev);
    int rc = expand(d, s);
    if (rc != OZ_OK) return rc;
    return rayleigh_ritz(d, d->xs[c ^ 1], s);
}

// step_tail from a captured graph (captured the first time c is seen), or
// issued directly when phases are being timed or graphs are off.
int run_tail(davidson d, int c, hipStream_t s) {
    hipError_t e;
    if (!d->use_graphs || d->ctx->timing) return step_tail(d, c, s);
    hipGraphExec_t &g = d->graphs[c];
    if (!g) {
        if (!d->cap && (e = hipStreamCreateWithFlags(&d->cap, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "davidson: capture stream");
        if ((e = hipStreamBeginCapture(d->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "davidson: begin capture");
        const int rc = step_tail(d, c, d->cap);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(d->cap, &graph);
        if (rc != OZ_OK) {
            if (graph) hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "davidson: end capture");
        e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g = nullptr;
            return hip_fail(e, "davidson: instantiate");
        }
    }
    if ((e = hipGraphLaunch(g, s)) != hipSuccess) return hip_fail(e, "davidson: graph launch");
    return OZ_OK;
}

}  // namespace

extern "C" {

int davidson_create(ozaki_ctx ctx, davidson *out, heff_plan H, const double *hdiag, const double *x0,
                    int m_max, double tol, int max_iter, void *stream) {
    if (!out) return fail(OZ_ERR_ARG, "davidson_create: out is NULL");
    *out = nullptr;
    if (!ctx || !H || !hdiag || !x0) return fail(OZ_ERR_ARG, "davidson_create: NULL argument");
    if (m_max < 2 || m_max > 64) return fail(OZ_ERR_ARG, "davidson_create: m_max = %d (2..64)", m_max);
    if (!(tol >= 0) || max_iter < 1) return fail(OZ_ERR_ARG, "davidson_create: tol / max_iter");
    const int64_t n = heff_vector_length(H);
    if (n < 1) return fail(OZ_ERR_ARG, "davidson_create: empty operator");
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    davidson d = new davidson_s();
    d->ctx = ctx;
    d->H = H;
    d->n = n;
    d->m_max = m_max;
    d->tol = tol;
    d->max_iter = max_iter;
    int rc;
    void *p;
#define OZ_DA(field, bytes) \
    if ((rc = dalloc(d, (bytes), &p)) != OZ_OK) { dfree(d); return rc; } \
    d->field = static_cast<std::remove_reference_t<decltype(d->field)>>(p);
    OZ_DA(V, sizeof(double) * m_max * n)
    OZ_DA(W, sizeof(double) * m_max * n)
    OZ_DA(G, sizeof(double) * m_max * m_max)
    OZ_DA(hdiag, sizeof(double) * n)
    OZ_DA(xs[0], sizeof(double) * n)
    OZ_DA(xs[1], sizeof(double) * n)
    OZ_DA(hx, sizeof(double) * n)
    OZ_DA(mv_in, sizeof(double) * n)
    OZ_DA(mv_out, sizeof(double) * n)
    OZ_DA(m_dev, sizeof(int) * 4)
    OZ_DA(r, sizeof(double) * n)
    OZ_DA(t, sizeof(double) * n)
    OZ_DA(y, sizeof(double) * 64)
    OZ_DA(coef, sizeof(double) * 64)
    OZ_DA(partial, sizeof(double) * 65 * 512)
    OZ_DA(scal, sizeof(double) * 8)
    OZ_DA(gate, sizeof(int) * 4)
#undef OZ_DA
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&d->host), sizeof(double) * 4, 0)) != hipSuccess) {
        d->host = nullptr;
        dfree(d);
        return hip_fail(e, "davidson_create: pinned buffer");
    }
    if ((e = hipMemcpyAsync(d->hdiag, hdiag, sizeof(double) * n, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemsetAsync(d->G, 0, sizeof(double) * m_max * m_max, s)) != hipSuccess) {
        dfree(d);
        return hip_fail(e, "davidson_create: copies");
    }
    // v0 = x0 / |x0|, W0 = H v0, G00 = v0 . W0
    double *nrm2 = d->scal + 2;
    if ((e = dots(d, x0, n, 1, x0, nrm2, 1, nullptr, 0, nullptr, s)) != hipSuccess ||
        (e = hipMemcpyAsync(d->host, nrm2, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        dfree(d);
        return hip_fail(e, "davidson_create: start vector");
    }
    if (!(d->host[0] > 0) || !std::isfinite(d->host[0])) {
        dfree(d);
        return fail(OZ_ERR_ARG, "davidson_create: start vector is zero or not finite");
    }
    hipLaunchKernelGGL(k_scale_into, dim3(grid_n(n)), dim3(256), 0, s, x0, nrm2, d->V, n);
    if ((rc = heff_apply(H, d->V, d->W, s)) != OZ_OK) { dfree(d); return rc; }
    dots(d, d->V, n, 1, d->W, d->G, 1, nullptr, 0, nullptr, s);
    const int one = 1;
    if ((e = hipMemcpyAsync(d->m_dev, &one, sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess) {
        dfree(d);
        return hip_fail(e, "davidson_create: basis size");
    }
    // the first step's Rayleigh-Ritz solve (every later one ends the step before)
    if ((rc = rayleigh_ritz(d, d->xs[0], s)) != OZ_OK) { dfree(d); return rc; }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { dfree(d); return hip_fail(e, "davidson_create: sync"); }
    d->m = 1;
    *out = d;
    return OZ_OK;
}

int davidson_step(davidson d, davidson_info *info, void *stream) {
    if (!d) return fail(OZ_ERR_ARG, "davidson_step: NULL solver");
    if (d->status != OZ_OK) {
        if (info) *info = davidson_info{d->host[0], std::sqrt(d->host[1]), d->iter, d->m, d->status};
        return fail(OZ_ERR_STATE, "davidson_step: the iteration has already ended (%s)", ozaki_status_string(d->status));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = hipSetDevice(d->ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    // the Rayleigh-Ritz solve on the current basis ended the previous step
    // (or davidson_create): its theta and rho^2 are in the pinned buffer
    d->iter += 1;
    const double theta = d->host[0];
    const double rho = std::sqrt(d->host[1]);
    d->hist.push_back(rho);
    d->rep = d->cur;
    int status = OZ_OK;
    const size_t w = 20;
    if (rho <= d->tol) {
        status = OZ_CONVERGED;
    } else if (d->hist.size() > w) {
        // stagnated: the last w residuals never got below half the best before them
        const size_t first_recent = d->hist.size() - w;
        double recent = INFINITY, before = INFINITY;
        for (size_t i = 0; i < d->hist.size(); ++i) {
            if (i >= first_recent)
                recent = std::min(recent, d->hist[i]);
            else
                before = std::min(before, d->hist[i]);
        }
        if (recent > 0.5 * before) status = OZ_STAGNATED;
    }
    if (status == OZ_OK && d->iter >= d->max_iter) status = OZ_MAX_ITER;
    if (status == OZ_OK) {
        // correction, basis update, matvec and the next Rayleigh-Ritz solve:
        // one graph replay and one synchronisation per step
        const int m = d->m;
        int rc = run_tail(d, d->cur, s);
        if (rc != OZ_OK) return rc;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "davidson_step: sync");
        d->m = (m == d->m_max ? 1 : m) + 1;
        d->cur ^= 1;
    }
    d->status = status;
    if (info) *info = davidson_info{theta, rho, d->iter, d->m, status};
    return status;
}

int davidson_set_graphs(davidson d, int enable) {
    if (!d) return fail(OZ_ERR_ARG, "davidson_set_graphs: NULL solver");
    d->use_graphs = enable != 0;
    return OZ_OK;
}

int davidson_graph_count(davidson d) {
    if (!d) return fail(OZ_ERR_ARG, "davidson_graph_count: NULL solver");
    int k = 0;
    for (auto g : d->graphs) k += g != nullptr;
    return k;
}

int davidson_get_vector(davidson d, double *x_out, void *stream) {
    if (!d || !x_out) return fail(OZ_ERR_ARG, "davidson_get_vector: NULL argument");
    if (d->iter == 0) return fail(OZ_ERR_STATE, "davidson_get_vector: no step taken yet");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(x_out, d->xs[d->rep], sizeof(double) * d->n, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? OZ_OK : hip_fail(e, "davidson_get_vector");
}

int davidson_destroy(davidson d) {
    if (!d) return OZ_OK;
    hipSetDevice(d->ctx->device);
    hipDeviceSynchronize();
    dfree(d);
    return OZ_OK;
}

}  // extern "C"

// ---- Lanczos with full reorthogonalisation and explicit restart -------------

namespace {

// x = Q^T y over the first m basis vectors.
__global__ void k_combine(const double *__restrict__ Q, int64_t n, int m, const double *__restrict__ y,
                          double *__restrict__ x) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s = fma(y[j], Q[j * n + i], s);
        x[i] = s;
    }
}

// Lowest eigenpair of the symmetric m x m matrix a (row-major), cyclic
// Jacobi on the host; y normalised with its largest-magnitude entry positive.
double host_lowest_eigenpair(std::vector<double> a, int m, std::vector<double> *y) {
    std::vector<double> v(static_cast<size_t>(m) * m, 0.0);
    for (int i = 0; i < m; ++i) v[static_cast<size_t>(i) * m + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                const double x = a[static_cast<size_t>(i) * m + j] * a[static_cast<size_t>(i) * m + j];
                tot += x;
                if (i != j) off += x;
            }
        if (std::sqrt(off) <= 1e-15 * std::sqrt(tot)) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = a[static_cast<size_t>(p) * m + q];
                if (apq == 0.0) continue;
                const double th = (a[static_cast<size_t>(q) * m + q] - a[static_cast<size_t>(p) * m + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {  // rows p, q
                    const double ap = a[static_cast<size_t>(p) * m + k], aq = a[static_cast<size_t>(q) * m + k];
                    a[static_cast<size_t>(p) * m + k] = c * ap - s * aq;
                    a[static_cast<size_t>(q) * m + k] = s * ap + c * aq;
                }
                for (int k = 0; k < m; ++k) {  // columns p, q and the eigenvectors
                    const double ap = a[static_cast<size_t>(k) * m + p], aq = a[static_cast<size_t>(k) * m + q];
                    a[static_cast<size_t>(k) * m + p] = c * ap - s * aq;
                    a[static_cast<size_t>(k) * m + q] = s * ap + c * aq;
                    const double vp = v[static_cast<size_t>(k) * m + p], vq = v[static_cast<size_t>(k) * m + q];
                    v[static_cast<size_t>(k) * m + p] = c * vp - s * vq;
                    v[static_cast<size_t>(k) * m + q] = s * vp + c * vq;
                }
            }
    }
    int best = 0;
    for (int i = 1; i < m; ++i)
        if (a[static_cast<size_t>(i) * m + i] < a[static_cast<size_t>(best) * m + best]) best = i;
    int big = 0;
    for (int i = 1; i < m; ++i)
        if (std::fabs(v[static_cast<size_t>(i) * m + best]) > std::fabs(v[static_cast<size_t>(big) * m + best])) big = i;
    const double sgn = v[static_cast<size_t>(big) * m + best] < 0 ? -1.0 : 1.0;
    y->resize(m);
    for (int i = 0; i < m; ++i) (*y)[i] = sgn * v[static_cast<size_t>(i) * m + best];
    return a[static_cast<size_t>(best) * m + best];
}

}  // namespace

struct lanczos_s {
    ozaki_ctx ctx = nullptr;
    heff_plan H = nullptr;
    int64_t n = 0;
    int m_max = 0, max_iter = 0;
    double tol = 0;
    std::vector<void *> allocs;
    double *Q = nullptr, *w = nullptr, *coef = nullptr, *partial = nullptr, *scal = nullptr, *y_dev = nullptr;
    int *gate = nullptr;
    double *host = nullptr;  // pinned: coefficients of the first pass, |w|^2
    std::vector<double> alpha, beta, y;
    int m = 0, iter = 0, status = OZ_OK;
    double theta = 0, rho = 0;
    std::vector<double> hist;
};

namespace {

int lalloc(lanczos l, size_t bytes, void **p) {
    hipError_t e = hipMalloc(p, bytes < 8 ? 8 : bytes);
    if (e != hipSuccess) return fail(OZ_ERR_NOMEM, "lanczos_create: %zu bytes: %s", bytes, hipGetErrorString(e));
    l->allocs.push_back(*p);
    return OZ_OK;
}

void lfree(lanczos l) {
    for (void *p : l->allocs) hipFree(p);
    if (l->host) hipHostFree(l->host);
    delete l;
}

// out[i] = Q_i . v for i < rows, with the Davidson dot kernels
hipError_t ldots(lanczos l, const double *Q, int rows, const double *v, double *out, hipStream_t s) {
    const int nb = dot_blocks(l->n);
    hipLaunchKernelGGL(k_dots_partial, dim3(nb, rows), dim3(kDotThreads), 0, s, Q, l->n, v, l->n, l->partial, nullptr,
                       DevRows{nullptr, 0});
    hipLaunchKernelGGL(k_dots_final, dim3(rows), dim3(kDotThreads), 0, s, l->partial, nb, out, 1, nullptr, 0, nullptr,
                       DevRows{nullptr, 0}, 0, 0);
    return hipGetLastError();
}

// q_0 = x / |x| into the basis; resets T
int lanczos_reset(lanczos l, const double *x, hipStream_t s) {
    hipError_t e;
    double *nrm2 = l->scal;
    if ((e = ldots(l, x, 1, x, nrm2, s)) != hipSuccess) return hip_fail(e, "lanczos: norm");
    hipLaunchKernelGGL(k_scale_into, dim3(grid_n(l->n)), dim3(256), 0, s, x, nrm2, l->Q, l->n);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "lanczos: normalise");
    l->m = 1;
    l->alpha.clear();
    l->beta.clear();
    return OZ_OK;
}

}  // namespace

extern "C" {

int lanczos_create(ozaki_ctx ctx, lanczos *out, heff_plan H, const double *x0, int m_max, double tol, int max_iter,
                   void *stream) {
    if (!out) return fail(OZ_ERR_ARG, "lanczos_create: out is NULL");
    *out = nullptr;
    if (!ctx || !H || !x0) return fail(OZ_ERR_ARG, "lanczos_create: NULL argument");
    if (m_max < 2 || m_max > 64) return fail(OZ_ERR_ARG, "lanczos_create: m_max = %d (2..64)", m_max);
    if (!(tol >= 0) || max_iter < 1) return fail(OZ_ERR_ARG, "lanczos_create: tol / max_iter");
    const int64_t n = heff_vector_length(H);
    if (n < 1) return fail(OZ_ERR_ARG, "lanczos_create: empty operator");
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    lanczos l = new lanczos_s();
    l->ctx = ctx;
    l->H = H;
    l->n = n;
    l->m_max = m_max;
    l->tol = tol;
    l->max_iter = max_iter;
    int rc;
    void *p;
#define OZ_LA(field, bytes) \
    if ((rc = lalloc(l, (bytes), &p)) != OZ_OK) { lfree(l); return rc; } \
    l->field = static_cast<decltype(l->field)>(p);
    OZ_LA(Q, sizeof(double) * (m_max + 1) * n)
    OZ_LA(w, sizeof(double) * n)
    OZ_LA(coef, sizeof(double) * 72)
    OZ_LA(partial, sizeof(double) * 66 * 512)
    OZ_LA(scal, sizeof(double) * 8)
    OZ_LA(y_dev, sizeof(double) * 72)
    OZ_LA(gate, sizeof(int) * 4)
#undef OZ_LA
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&l->host), sizeof(double) * 72, 0)) != hipSuccess) {
        l->host = nullptr;
        lfree(l);
        return hip_fail(e, "lanczos_create: pinned buffer");
    }
    // start vector: |x0| must be positive and finite
    if ((e = ldots(l, x0, 1, x0, l->scal, s)) != hipSuccess ||
        (e = hipMemcpyAsync(l->host, l->scal, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        lfree(l);
        return hip_fail(e, "lanczos_create: start vector");
    }
    if (!(l->host[0] > 0) || !std::isfinite(l->host[0])) {
        lfree(l);
        return fail(OZ_ERR_ARG, "lanczos_create: start vector is zero or not finite");
    }
    if ((rc = lanczos_reset(l, x0, s)) != OZ_OK) { lfree(l); return rc; }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { lfree(l); return hip_fail(e, "lanczos_create: sync"); }
    *out = l;
    return OZ_OK;
}

int lanczos_step(lanczos l, davidson_info *info, void *stream) {
    if (!l) return fail(OZ_ERR_ARG, "lanczos_step: NULL solver");
    if (l->status != OZ_OK) {
        if (info) *info = davidson_info{l->theta, l->rho, l->iter, l->m, l->status};
        return fail(OZ_ERR_STATE, "lanczos_step: the iteration has already ended (%s)", ozaki_status_string(l->status));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = hipSetDevice(l->ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    const int64_t n = l->n;
    const int m = l->m;  // basis q_0 .. q_{m-1}; this step expands from q_{m-1}
    double *qj = l->Q + static_cast<int64_t>(m - 1) * n;
    int rc = heff_apply(l->H, qj, l->w, s);
    if (rc != OZ_OK) return rc;
    // two classical Gram-Schmidt passes against the whole basis; alpha from the first
    for (int pass = 0; pass < 2; ++pass) {
        if ((e = ldots(l, l->Q, m, l->w, l->coef, s)) != hipSuccess) return hip_fail(e, "lanczos: projection");
        if (pass == 0 && (e = hipMemcpyAsync(l->host, l->coef, sizeof(double) * m, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "lanczos: coefficients");
        hipLaunchKernelGGL(k_project, dim3(grid_n(n)), dim3(256), 0, s, l->Q, n, m, nullptr, l->coef, l->w, nullptr);
    }
    if ((e = ldots(l, l->w, 1, l->w, l->scal, s)) != hipSuccess) return hip_fail(e, "lanczos: norm");
    if ((e = hipMemcpyAsync(l->host + 64, l->scal, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "lanczos: step");
    l->iter += 1;
    const double a = l->host[m - 1];
    const double b = std::sqrt(l->host[64] > 0 ? l->host[64] : 0.0);
    l->alpha.push_back(a);
    // Ritz pair of T_m
    std::vector<double> T(static_cast<size_t>(m) * m, 0.0);
    for (int i = 0; i < m; ++i) {
        T[static_cast<size_t>(i) * m + i] = l->alpha[i];
        if (i + 1 < m) T[static_cast<size_t>(i) * m + i + 1] = T[static_cast<size_t>(i + 1) * m + i] = l->beta[i];
    }
    l->theta = host_lowest_eigenpair(T, m, &l->y);
    l->rho = b * std::fabs(l->y[m - 1]);
    l->hist.push_back(l->rho);
    int status = OZ_OK;
    const bool invariant = !(b > 1e-14 * (std::fabs(a) + (m > 1 ? l->beta[m - 2] : 0.0)));
    if (l->rho <= l->tol || invariant) {
        status = OZ_CONVERGED;
    } else if (l->hist.size() > 20) {
        const size_t first_recent = l->hist.size() - 20;
        double recent = INFINITY, before = INFINITY;
        for (size_t i = 0; i < l->hist.size(); ++i) {
            if (i >= first_recent) recent = std::min(recent, l->hist[i]);
            else before = std::min(before, l->hist[i]);
        }
        if (recent > 0.5 * before) status = OZ_STAGNATED;
    }
    if (status == OZ_OK && l->iter >= l->max_iter) status = OZ_MAX_ITER;
    if (status == OZ_OK) {
        if (m == l->m_max) {
            // restart from the Ritz vector x = Q y (written to w, then normalised into q_0)
            if ((e = hipMemcpyAsync(l->y_dev, l->y.data(), sizeof(double) * m, hipMemcpyHostToDevice, s)) != hipSuccess)
                return hip_fail(e, "lanczos: Ritz coefficients");
            hipLaunchKernelGGL(k_combine, dim3(grid_n(n)), dim3(256), 0, s, l->Q, n, m, l->y_dev, l->w);
            if ((rc = lanczos_reset(l, l->w, s)) != OZ_OK) return rc;
        } else {
            l->beta.push_back(b);
            hipLaunchKernelGGL(k_scale_into, dim3(grid_n(n)), dim3(256), 0, s, l->w, l->scal,
                               l->Q + static_cast<int64_t>(m) * n, n);
            if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "lanczos: expand");
            l->m = m + 1;
        }
    } else {
        // keep the Ritz coefficients of the final basis for lanczos_get_vector
        l->m = m;
    }
    l->status = status;
    if (info) *info = davidson_info{l->theta, l->rho, l->iter, l->m, status};
    return status;
}

int lanczos_get_vector(lanczos l, double *x_out, void *stream) {
    if (!l || !x_out) return fail(OZ_ERR_ARG, "lanczos_get_vector: NULL argument");
    if (l->iter == 0 || l->y.empty()) return fail(OZ_ERR_STATE, "lanczos_get_vector: no step taken yet");
    if (l->status == OZ_OK && l->m == 1 && l->alpha.empty()) {
        // just restarted: q_0 is the Ritz vector
        hipError_t e = hipMemcpyAsync(x_out, l->Q, sizeof(double) * l->n, hipMemcpyDeviceToDevice,
                                      static_cast<hipStream_t>(stream));
        return e == hipSuccess ? OZ_OK : hip_fail(e, "lanczos_get_vector");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int m = static_cast<int>(l->y.size());
    hipError_t e = hipMemcpyAsync(l->y_dev, l->y.data(), sizeof(double) * m, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "lanczos_get_vector: coefficients");
    hipLaunchKernelGGL(k_combine, dim3(grid_n(l->n)), dim3(256), 0, s, l->Q, l->n, m, l->y_dev, x_out);
    e = hipStreamSynchronize(s);  // y_dev is reused by the next step
    return e == hipSuccess ? OZ_OK : hip_fail(e, "lanczos_get_vector");
}

int lanczos_destroy(lanczos l) {
    if (!l) return OZ_OK;
    hipSetDevice(l->ctx->device);
    hipDeviceSynchronize();
    lfree(l);
    return OZ_OK;
}

}  // extern "C"
