// Steps 1 and 2 of the emulated GEMM ("Theory of emulated FP64 arithmetic"):
// one power-of-two exponent per row of A / column of B, then S balanced
// int8 slices per element, written in the packed layout of internal.h.
//
// All three kernels are HBM-bound: the exponent pass reads X once (8 B per
// element); the slice pass reads it again and writes S bytes per element.
#include "internal.h"

namespace oz {
namespace {

// |x| for a finite x, NaN for NaN or +-Inf (marks the group as non-finite).
__device__ inline double abs_or_nan(double x) {
    if (!(fabs(x) <= 1.79769313486231570815e308)) return __longlong_as_double(0x7ff8000000000000ll);
    return fabs(x);
}

// Maximum that propagates NaN from either side.
__device__ inline double combine_max(double a, double b) {
    if (a != a || b != b) return __longlong_as_double(0x7ff8000000000000ll);
    return a > b ? a : b;
}

__device__ inline int32_t finish_exponent(double mu, uint32_t *flag) {
    if (mu != mu) {
        atomicOr(flag, 1u);
        return kExpBad;
    }
    return shared_exponent(mu);
}

// One wave per row; 4 rows per 256-thread block.
__global__ __launch_bounds__(256) void k_row_exponents(const double *__restrict__ X, int64_t ld,
                                                        int64_t R, int64_t K,
                                                        int32_t *__restrict__ e,
                                                        uint32_t *flag) {
    const int lane = threadIdx.x & 63;
    const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (r >= R) return;
    const double *row = X + r * ld;
    // four loads in flight per lane; the maximum does not depend on the order
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    int64_t k = lane;
    for (; k + 192 < K; k += 256) {
        const double a = row[k], b = row[k + 64], c = row[k + 128], d = row[k + 192];
        m0 = combine_max(m0, abs_or_nan(a));
        m1 = combine_max(m1, abs_or_nan(b));
        m2 = combine_max(m2, abs_or_nan(c));
        m3 = combine_max(m3, abs_or_nan(d));
    }
    for (; k < K; k += 64) m0 = combine_max(m0, abs_or_nan(row[k]));
    double mu = combine_max(combine_max(m0, m1), combine_max(m2, m3));
    for (int off = 32; off >= 1; off >>= 1) mu = combine_max(mu, __shfl_xor(mu, off, 64));
    if (lane == 0) e[r] = finish_exponent(mu, flag);
}

// Column maxima of X (K x R): block (column strip of 256, row chunk of 256).
constexpr int kColChunk = 256;

__global__ __launch_bounds__(256) void k_col_partial(const double *__restrict__ X, int64_t ld,
                                                      int64_t K, int64_t R,
                                                      double *__restrict__ part) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (c >= R) return;
    const int64_t k0 = static_cast<int64_t>(blockIdx.y) * kColChunk;
    const int64_t k1 = k0 + kColChunk < K ? k0 + kColChunk : K;
    // eight loads in flight per lane; the maximum does not depend on the order
    double m[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t k = k0;
    for (; k + 8 <= k1; k += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = X[(k + q) * ld + c];
#pragma unroll
        for (int q = 0; q < 8; ++q) m[q] = combine_max(m[q], abs_or_nan(v[q]));
    }
    for (; k < k1; ++k) m[0] = combine_max(m[0], abs_or_nan(X[k * ld + c]));
    double mu = m[0];
#pragma unroll
    for (int q = 1; q < 8; ++q) mu = combine_max(mu, m[q]);
    part[static_cast<int64_t>(blockIdx.y) * R + c] = mu;
}

__global__ __launch_bounds__(256) void k_col_final(const double *__restrict__ part, int64_t nchunk,
                                                    int64_t R, int32_t *__restrict__ e,
                                                    uint32_t *flag) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (c >= R) return;
    double mu = 0.0;
    for (int64_t q = 0; q < nchunk; ++q) mu = combine_max(mu, part[q * R + c]);
    e[c] = finish_exponent(mu, flag);
}

// Sums of squares per group (statistics of the automatic slice count).
// Rows: one wave per row, lanes stride the row, fixed shuffle tree.
__global__ __launch_bounds__(256) void k_row_sumsq(const double *__restrict__ X, int64_t ld, int64_t R,
                                                    int64_t K, double *__restrict__ ss) {
    const int lane = threadIdx.x & 63;
    const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (r >= R) return;
    const double *row = X + r * ld;
    double acc = 0.0;
    for (int64_t k = lane; k < K; k += 64) acc = fma(row[k], row[k], acc);
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) ss[r] = acc;
}

// Columns of X (K x R): partial sums over row chunks, then the chunks in order.
__global__ __launch_bounds__(256) void k_col_sumsq_partial(const double *__restrict__ X, int64_t ld,
                                                            int64_t K, int64_t R, double *__restrict__ part) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (c >= R) return;
    const int64_t k0 = static_cast<int64_t>(blockIdx.y) * kColChunk;
    const int64_t k1 = k0 + kColChunk < K ? k0 + kColChunk : K;
    double acc = 0.0;
    for (int64_t k = k0; k < k1; ++k) {
        const double x = X[k * ld + c];
        acc = fma(x, x, acc);
    }
    part[static_cast<int64_t>(blockIdx.y) * R + c] = acc;
}

__global__ __launch_bounds__(256) void k_col_sumsq_final(const double *__restrict__ part, int64_t nchunk,
                                                          int64_t R, double *__restrict__ ss) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (c >= R) return;
    double acc = 0.0;
    for (int64_t q = 0; q < nchunk; ++q) acc += part[q * R + c];
    ss[c] = acc;
}

// Balanced base-256 digits of one element, most significant first.
template <int S>
__device__ inline void digits(double x, int32_t e, int (&d)[S]) {
    long long X = static_cast<long long>(rint(ldexp(x, 8 * S - 1 - e)));
#pragma unroll
    for (int t = S - 1; t >= 1; --t) {
        d[t] = static_cast<int>((X + 128) & 255) - 128;
        X = (X - d[t]) >> 8;
    }
    d[0] = static_cast<int>(X);
}

// Balanced base-256 digits of RNE(x 2^(8S-1-e)), most significant first, as
// bytes of four consecutive elements packed into one word per slice.
template <int S>
__device__ inline void slice4(const double (&x)[4], int32_t e, uint32_t (&w)[S]) {
#pragma unroll
    for (int s = 0; s < S; ++s) w[s] = 0;
    if (e == kExpBad) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        long long X = static_cast<long long>(rint(ldexp(x[q], 8 * S - 1 - e)));
        int d[S];
#pragma unroll
        for (int t = S - 1; t >= 1; --t) {
            d[t] = static_cast<int>((X + 128) & 255) - 128;
            X = (X - d[t]) >> 8;
        }
        d[0] = static_cast<int>(X);
#pragma unroll
        for (int s = 0; s < S; ++s) w[s] |= (static_cast<uint32_t>(d[s]) & 0xffu) << (8 * q);
    }
}

// 32 groups x 32 inner elements per block.  TRANS = false: X is R x K and a
// group is a row; TRANS = true: X is K x R and a group is a column.
template <int S, bool TRANS>
__global__ __launch_bounds__(256) void k_slice(const double *__restrict__ X, int64_t ld, int64_t R,
                                                int64_t K, const int32_t *__restrict__ e,
                                                int8_t *__restrict__ packed, int64_t Rp) {
    __shared__ uint4 tile[S * 2][32];
    const int t = threadIdx.x;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * 32;
    const int64_t kb = blockIdx.y;
    const int64_t k0 = kb * 32;
    if (TRANS) {
        // lanes take consecutive groups (columns): every load is coalesced
        const int r = t & 31, kq = t >> 5;
        const int64_t gr = r0 + r;
        double x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t k = k0 + kq * 4 + q;
            x[q] = (gr < R && k < K) ? X[k * ld + gr] : 0.0;
        }
        uint32_t w[S];
        slice4<S>(x, gr < R ? e[gr] : 0, w);
        const int c = kq >> 2, word = kq & 3;
#pragma unroll
        for (int s = 0; s < S; ++s) reinterpret_cast<uint32_t *>(&tile[s * 2 + c][r])[word] = w[s];
    } else {
        // 16 lanes per row, two consecutive elements each (one 16-byte load
        // when the block is whole and aligned), rows r and r + 16; the two
        // bytes per slice of a lane pair make one word of the tile
        const int kp = t & 15;
        const bool full = r0 + 32 <= R && k0 + 32 <= K && (ld & 1) == 0 &&
                          (reinterpret_cast<uintptr_t>(X) & 15) == 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = (t >> 4) + 16 * h;
            const int64_t gr = r0 + r;
            const int64_t k = k0 + 2 * kp;
            double x0 = 0.0, x1 = 0.0;
            if (full) {
                const double2 v = *reinterpret_cast<const double2 *>(X + gr * ld + k);
                x0 = v.x;
                x1 = v.y;
            } else if (gr < R) {
                if (k < K) x0 = X[gr * ld + k];
                if (k + 1 < K) x1 = X[gr * ld + k + 1];
            }
            const int32_t ee = gr < R ? e[gr] : 0;
            uint32_t half[S];
#pragma unroll
            for (int s = 0; s < S; ++s) half[s] = 0;
            if (ee != kExpBad) {
                int d0[S], d1[S];
                digits<S>(x0, ee, d0);
                digits<S>(x1, ee, d1);
#pragma unroll
                for (int s = 0; s < S; ++s)
                    half[s] = (static_cast<uint32_t>(d0[s]) & 0xffu) | ((static_cast<uint32_t>(d1[s]) & 0xffu) << 8);
            }
            const int kq = kp >> 1, c = kq >> 2, word = kq & 3;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const uint32_t other = static_cast<uint32_t>(__shfl_down(static_cast<int>(half[s]), 1, 64));
                if ((kp & 1) == 0)
                    reinterpret_cast<uint32_t *>(&tile[s * 2 + c][r])[word] = half[s] | (other << 16);
            }
        }
    }
    __syncthreads();
    // write 2S runs of 32 rows x 16 bytes
    uint4 *out = reinterpret_cast<uint4 *>(packed);
    for (int q = t; q < S * 2 * 32; q += 256) {
        const int sc = q >> 5;
        const int rr = q & 31;
        out[(kb * S * 2 + sc) * Rp + r0 + rr] = tile[sc][rr];
    }
}

template <int S>
hipError_t slice_s(bool trans, const double *X, int64_t ld, int64_t R, int64_t K,
                   const int32_t *e, int8_t *packed, int64_t Rp, hipStream_t s) {
    dim3 grid(static_cast<unsigned>(Rp / 32), static_cast<unsigned>(ceil_div(K, kKB)));
    if (trans)
        hipLaunchKernelGGL((k_slice<S, true>), grid, dim3(256), 0, s, X, ld, R, K, e, packed, Rp);
    else
        hipLaunchKernelGGL((k_slice<S, false>), grid, dim3(256), 0, s, X, ld, R, K, e, packed, Rp);
    return hipGetLastError();
}

// ---- grouped versions: one launch for a list of blocks -------------------
// Row groups (trans = 0): 16 rows per task, four per wave, the loads of the
// four rows interleaved so each lane keeps several in flight.
// Column groups (trans = 1): 64 columns per task, one per lane; the four
// waves take every fourth row of the block, eight loads in flight per lane,
// and combine their maxima through LDS.  The maximum is order independent
// (NaN wins), so the split does not change the exponents.

__global__ __launch_bounds__(256) void k_exponents_grouped(const SliceBlock *__restrict__ blocks,
                                                            const SliceTask *__restrict__ tasks,
                                                            const double *__restrict__ x_base,
                                                            int32_t *__restrict__ e_base,
                                                            uint32_t *flag, int32_t *emax_base) {
    __shared__ double part[4][kExpTaskCols];
    const SliceTask tk = tasks[blockIdx.x];
    const SliceBlock bl = blocks[tk.block];
    const double *X = x_base + bl.x_off;
    int32_t *e = e_base + bl.e_off;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (bl.trans == 0) {
        const int r0 = tk.a + wave * 4;
        double mu[4] = {0.0, 0.0, 0.0, 0.0};
        const double *row[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) row[j] = X + static_cast<int64_t>(r0 + j < bl.R ? r0 + j : 0) * bl.ld;
        // two elements of each of the 4 rows per iteration: 8 loads in flight per lane
        int k = lane;
        for (; k + 64 < bl.K; k += 128) {
            double v[4][2];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool ok = r0 + j < bl.R;
                v[j][0] = ok ? row[j][k] : 0.0;
                v[j][1] = ok ? row[j][k + 64] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                mu[j] = combine_max(mu[j], combine_max(abs_or_nan(v[j][0]), abs_or_nan(v[j][1])));
        }
        if (k < bl.K) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (r0 + j < bl.R) mu[j] = combine_max(mu[j], abs_or_nan(row[j][k]));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double m = mu[j];
            for (int off = 32; off >= 1; off >>= 1) m = combine_max(m, __shfl_xor(m, off, 64));
            if (lane == 0 && r0 + j < bl.R) {
                if (!emax_base)
                    e[r0 + j] = finish_exponent(m, flag);
                else if (m != 0.0)
                    atomicMax(emax_base + bl.e_off + r0 + j, m != m ? kEmaxNaN : shared_exponent(m));
            }
        }
    } else {
        const int c = tk.a + lane;
        const bool cok = c < bl.R;
        const double *col = X + (cok ? c : 0);
        // rows [k0, k1): all of them, or one chunk of a split column task
        const int k0 = emax_base ? tk.b * kExpColChunk : 0;
        const int k1 = emax_base ? min(bl.K, k0 + kExpColChunk) : bl.K;
        double m8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) m8[u] = 0.0;
        int k = k0 + wave;
        for (; k + 28 < k1; k += 32) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                m8[u] = combine_max(m8[u], cok ? abs_or_nan(col[static_cast<int64_t>(k + 4 * u) * bl.ld]) : 0.0);
        }
        for (; k < k1; k += 4) m8[0] = combine_max(m8[0], cok ? abs_or_nan(col[static_cast<int64_t>(k) * bl.ld]) : 0.0);
        double mu = m8[0];
#pragma unroll
        for (int u = 1; u < 8; ++u) mu = combine_max(mu, m8[u]);
        part[wave][lane] = mu;
        __syncthreads();
        if (wave == 0) {
            mu = combine_max(combine_max(part[0][lane], part[1][lane]), combine_max(part[2][lane], part[3][lane]));
            if (cok) {
                if (!emax_base) {
                    e[c] = finish_exponent(mu, flag);
                } else if (mu != 0.0) {
                    // the code is monotone in the magnitude: the chunks' largest code is the column's
                    atomicMax(emax_base + bl.e_off + c, mu != mu ? kEmaxNaN : shared_exponent(mu));
                }
            }
        }
    }
}

// Exponents from the maxima a producing GEMM left in emax (one code per
// group, combined with atomic max): the code itself, 0 for an all-zero
// group, kExpBad and the flag for a non-finite one.  emax is reset to
// kEmaxZero for the next product.
__global__ __launch_bounds__(256) void k_emax_finish(int32_t *__restrict__ emax, int32_t *__restrict__ e,
                                                      int64_t n, uint32_t *flag) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        const int32_t v = emax[i];
        int32_t x = v;
        if (v == kEmaxNaN) {
            atomicOr(flag, 1u);
            x = kExpBad;
        } else if (v == kEmaxZero) {
            x = 0;
        }
        e[i] = x;
        emax[i] = kEmaxZero;
    }
}

// One task: 32 groups x up to kSliceTaskKB consecutive 32-wide K blocks; the
// elements of the next K block are loaded while the current one is sliced.

template <int S>
__global__ __launch_bounds__(256) void k_slice_grouped(const SliceBlock *__restrict__ blocks,
                                                        const SliceTask *__restrict__ tasks,
                                                        const double *__restrict__ x_base,
                                                        const int32_t *__restrict__ e_base,
                                                        int8_t *__restrict__ p_base) {
    __shared__ uint4 tile[S * 2][32];
    const SliceTask tk = tasks[blockIdx.x];
    const SliceBlock bl = blocks[tk.block];
    const double *X = x_base + bl.x_off;
    const int32_t *e = e_base + bl.e_off;
    const int t = threadIdx.x;
    const int64_t r0 = tk.a;
    const int nkb = (bl.K + kKB - 1) / kKB;
    const int kb_end = tk.b + kSliceTaskKB < nkb ? tk.b + kSliceTaskKB : nkb;
    uint4 *out = reinterpret_cast<uint4 *>(p_base + bl.p_off);
    auto flush = [&](int kb) {
        __syncthreads();
        for (int q = t; q < S * 2 * 32; q += 256) {
            const int sc = q >> 5;
            const int rr = q & 31;
            out[(static_cast<int64_t>(kb) * S * 2 + sc) * bl.Rp + r0 + rr] = tile[sc][rr];
        }
        __syncthreads();
    };
    if (bl.trans) {
        // lanes take consecutive groups (columns): every load is coalesced
        const int r = t & 31, kq = t >> 5;
        const int64_t gr = r0 + r;
        const int32_t ee = gr < bl.R ? e[gr] : 0;
        auto load = [&](int kb, double (&x)[4]) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t k = static_cast<int64_t>(kb) * 32 + kq * 4 + q;
                x[q] = (gr < bl.R && k < bl.K) ? X[k * bl.ld + gr] : 0.0;
            }
        };
        double x[4], nx[4];
        load(tk.b, x);
        const int c = kq >> 2, word = kq & 3;
        for (int kb = tk.b; kb < kb_end; ++kb) {
            if (kb + 1 < kb_end) load(kb + 1, nx);
            uint32_t w[S];
            slice4<S>(x, ee, w);
#pragma unroll
            for (int s = 0; s < S; ++s) reinterpret_cast<uint32_t *>(&tile[s * 2 + c][r])[word] = w[s];
            flush(kb);
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = nx[q];
        }
        return;
    }
    // row groups: 16 lanes per row, two consecutive elements each (one
    // 16-byte load when aligned and inside the block), rows r and r + 16;
    // the two bytes per slice of a lane pair make one word of the tile
    const int kp = t & 15;
    const int rA = t >> 4;
    const bool aligned = (bl.ld & 1) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
    int32_t ee[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) ee[h] = r0 + rA + 16 * h < bl.R ? e[r0 + rA + 16 * h] : 0;
    auto load = [&](int kb, double (&x)[4]) {
        const int64_t k = static_cast<int64_t>(kb) * 32 + 2 * kp;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t gr = r0 + rA + 16 * h;
            x[2 * h] = 0.0;
            x[2 * h + 1] = 0.0;
            if (gr < bl.R) {
                if (aligned && k + 1 < bl.K) {
                    const double2 v = *reinterpret_cast<const double2 *>(X + gr * bl.ld + k);
                    x[2 * h] = v.x;
                    x[2 * h + 1] = v.y;
                } else {
                    if (k < bl.K) x[2 * h] = X[gr * bl.ld + k];
                    if (k + 1 < bl.K) x[2 * h + 1] = X[gr * bl.ld + k + 1];
                }
            }
        }
    };
    double x[4], nx[4];
    load(tk.b, x);
    const int kq = kp >> 1, c = kq >> 2, word = kq & 3;
    for (int kb = tk.b; kb < kb_end; ++kb) {
        if (kb + 1 < kb_end) load(kb + 1, nx);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t half[S];
#pragma unroll
            for (int s = 0; s < S; ++s) half[s] = 0;
            if (ee[h] != kExpBad) {
                int d0[S], d1[S];
                digits<S>(x[2 * h], ee[h], d0);
                digits<S>(x[2 * h + 1], ee[h], d1);
#pragma unroll
                for (int s = 0; s < S; ++s)
                    half[s] = (static_cast<uint32_t>(d0[s]) & 0xffu) | ((static_cast<uint32_t>(d1[s]) & 0xffu) << 8);
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const uint32_t other = static_cast<uint32_t>(__shfl_down(static_cast<int>(half[s]), 1, 64));
                if ((kp & 1) == 0)
                    reinterpret_cast<uint32_t *>(&tile[s * 2 + c][rA + 16 * h])[word] = half[s] | (other << 16);
            }
        }
        flush(kb);
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = nx[q];
    }
}

// Debug layout conversions, one byte per thread.
__global__ void k_pack(int S, const int8_t *__restrict__ canon, int64_t R, int64_t K,
                       int8_t *__restrict__ packed, int64_t Rp, int64_t Kp) {
    const int64_t total = static_cast<int64_t>(S) * Rp * Kp;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t s = i / (Rp * Kp);
        const int64_t r = (i / Kp) % Rp;
        const int64_t k = i % Kp;
        const int8_t v = (r < R && k < K) ? canon[(s * R + r) * K + k] : int8_t(0);
        packed[((k / 32 * S + s) * 2 + (k / 16) % 2) * Rp * 16 + r * 16 + k % 16] = v;
    }
}

__global__ void k_unpack(int S, const int8_t *__restrict__ packed, int64_t Rp, int64_t R,
                         int64_t K, int8_t *__restrict__ canon) {
    const int64_t total = static_cast<int64_t>(S) * R * K;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t s = i / (R * K);
        const int64_t r = (i / K) % R;
        const int64_t k = i % K;
        canon[i] = packed[((k / 32 * S + s) * 2 + (k / 16) % 2) * Rp * 16 + r * 16 + k % 16];
    }
}

__global__ void k_diag_axpy(const double *__restrict__ diag, const double *__restrict__ psi,
                            double *__restrict__ sigma, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double p = diag[i] * psi[i];
        sigma[i] = sigma[i] + p;
    }
}

unsigned grid_for(int64_t n, int64_t per_block, unsigned cap) {
    const int64_t g = ceil_div(n, per_block);
    return static_cast<unsigned>(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_row_exponents(const double *X, int64_t ld, int64_t R, int64_t K, int32_t *e,
                                uint32_t *flag, hipStream_t s) {
    if (R == 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_exponents, dim3(static_cast<unsigned>(ceil_div(R, 4))), dim3(256), 0,
                       s, X, ld, R, K, e, flag);
    return hipGetLastError();
}

size_t col_exponent_scratch(int64_t K, int64_t R) {
    const int64_t nchunk = ceil_div(K, kColChunk) < 1 ? 1 : ceil_div(K, kColChunk);
    return static_cast<size_t>(nchunk * R) * sizeof(double);
}

hipError_t launch_col_exponents(const double *X, int64_t ld, int64_t K, int64_t R, int32_t *e,
                                double *part, uint32_t *flag, hipStream_t s) {
    if (R == 0) return hipSuccess;
    const int64_t nchunk = ceil_div(K, kColChunk);
    if (nchunk > 0) {
        hipLaunchKernelGGL(k_col_partial,
                           dim3(static_cast<unsigned>(ceil_div(R, 256)), static_cast<unsigned>(nchunk)),
                           dim3(256), 0, s, X, ld, K, R, part);
    }
    hipLaunchKernelGGL(k_col_final, dim3(static_cast<unsigned>(ceil_div(R, 256))), dim3(256), 0, s,
                       part, nchunk, R, e, flag);
    return hipGetLastError();
}

hipError_t launch_group_sumsq(bool by_rows, const double *X, int64_t ld, int64_t R, int64_t K, double *ss,
                              double *part, hipStream_t s) {
    if (R == 0) return hipSuccess;
    if (by_rows) {
        hipLaunchKernelGGL(k_row_sumsq, dim3(static_cast<unsigned>(ceil_div(R, 4))), dim3(256), 0, s, X, ld, R, K, ss);
        return hipGetLastError();
    }
    const int64_t nchunk = ceil_div(K, kColChunk);
    if (nchunk > 0)
        hipLaunchKernelGGL(k_col_sumsq_partial,
                           dim3(static_cast<unsigned>(ceil_div(R, 256)), static_cast<unsigned>(nchunk)), dim3(256), 0, s,
                           X, ld, K, R, part);
    hipLaunchKernelGGL(k_col_sumsq_final, dim3(static_cast<unsigned>(ceil_div(R, 256))), dim3(256), 0, s, part, nchunk,
                       R, ss);
    return hipGetLastError();
}

hipError_t launch_slice(int S, bool trans, const double *X, int64_t ld, int64_t R, int64_t K,
                        const int32_t *e, int8_t *packed, int64_t Rp, hipStream_t s) {
    if (Rp == 0 || K == 0) return hipSuccess;
    switch (S) {
        case 2: return slice_s<2>(trans, X, ld, R, K, e, packed, Rp, s);
        case 3: return slice_s<3>(trans, X, ld, R, K, e, packed, Rp, s);
        case 4: return slice_s<4>(trans, X, ld, R, K, e, packed, Rp, s);
        case 5: return slice_s<5>(trans, X, ld, R, K, e, packed, Rp, s);
        case 6: return slice_s<6>(trans, X, ld, R, K, e, packed, Rp, s);
        case 7: return slice_s<7>(trans, X, ld, R, K, e, packed, Rp, s);
        case 8: return slice_s<8>(trans, X, ld, R, K, e, packed, Rp, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_exponents_grouped(const SliceBlock *blocks, const SliceTask *tasks, int ntasks,
                                    const double *x_base, int32_t *e_base, uint32_t *flag,
                                    hipStream_t s, int32_t *emax_base) {
    if (ntasks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_exponents_grouped, dim3(ntasks), dim3(256), 0, s, blocks, tasks, x_base,
                       e_base, flag, emax_base);
    return hipGetLastError();
}

hipError_t launch_emax_finish(int32_t *emax, int32_t *e, int64_t n, uint32_t *flag, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_emax_finish, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, emax, e, n, flag);
    return hipGetLastError();
}

hipError_t launch_slice_grouped(int S, const SliceBlock *blocks, const SliceTask *tasks, int ntasks,
                                const double *x_base, const int32_t *e_base, int8_t *p_base,
                                hipStream_t s) {
    if (ntasks == 0) return hipSuccess;
#define OZ_SG(S_)                                                                                \
    case S_:                                                                                     \
        hipLaunchKernelGGL(k_slice_grouped<S_>, dim3(ntasks), dim3(256), 0, s, blocks, tasks,    \
                           x_base, e_base, p_base);                                             \
        break;
    switch (S) {
        OZ_SG(2) OZ_SG(3) OZ_SG(4) OZ_SG(5) OZ_SG(6) OZ_SG(7) OZ_SG(8)
        default: return hipErrorInvalidValue;
    }
#undef OZ_SG
    return hipGetLastError();
}

hipError_t launch_pack(int S, const int8_t *canon, int64_t R, int64_t K, int8_t *packed,
                       int64_t Rp, hipStream_t s) {
    const int64_t Kp = round_up(K, kKB);
    const int64_t total = static_cast<int64_t>(S) * Rp * Kp;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3(grid_for(total, 256, 65535)), dim3(256), 0, s, S, canon, R, K,
                       packed, Rp, Kp);
    return hipGetLastError();
}

hipError_t launch_unpack(int S, const int8_t *packed, int64_t Rp, int64_t R, int64_t K,
                         int8_t *canon, hipStream_t s) {
    const int64_t total = static_cast<int64_t>(S) * R * K;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpack, dim3(grid_for(total, 256, 65535)), dim3(256), 0, s, S, packed, Rp,
                       R, K, canon);
    return hipGetLastError();
}

hipError_t launch_diag_axpy(const double *diag, const double *psi, double *sigma, int64_t n,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag_axpy, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, diag, psi,
                       sigma, n);
    return hipGetLastError();
}

}  // namespace oz
