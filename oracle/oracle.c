/*
 * CPU oracle for Ozaki-scheme emulated DGEMM (slices of int8 fixed point).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the HIP library.
 *
 * Plain, slow and meant to be checked by eye against the paper
 * ("Theory of emulated FP64 arithmetic", four-step strategy):
 *   step 1  fixed point with an exponent shared per row of A / column of B
 *   step 2  split into S low-precision slices A^i, B^j
 *   step 3  every slice pair (i, j) multiplied on its own, exactly
 *   step 4  products accumulated and converted back to FP64
 * together with the slice count <-> mantissa bit rule of "Numerical
 * procedure" (S = ceildiv(bits + 1, 8), i.e. 8S - 1 magnitude bits + sign).
 *
 * Where the paper is silent the oracle follows these readings:
 *   exponent  e = E + [m > 127/128] with (m, E) = frexp(max |x|), 0 for a
 *             zero row, so the leading slice fits in int8;
 *   rounding  X = RNE(x * 2^(8S-1-e)) (exact scaling, one rounding);
 *   digits    balanced base-256: X = sum_t d_t 256^(S-1-t), d_t in
 *             [-128, 127] for t >= 1, |d_0| <= 127;
 *   pairs     kept pairs are those with s + t < G (G = S drops the
 *             less-significant lower triangle; G = 2S - 1 keeps all S^2);
 *   recombine h = Q_{G-1}; h = h * 2^-8 + Q_g for g = G-2 .. 0 (one FP64
 *             rounding per step), c = h * 2^(e_i + f_j - 14);
 *   output    C = alpha * c if beta == 0, else fma(alpha, c, beta * C);
 *             a row/column holding NaN or Inf gives a NaN row/column.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------
 * Plain FP64 GEMM: c_ij = sum_k a_ik b_kj, k ascending, one fma per term.
 * C = alpha * c (beta == 0, C not read) or fma(alpha, c, beta * C).
 * Any summation order is an equally valid FP64 GEMM; this one is the
 * textbook loop, bounded by gamma_K |A||B| (Higham, ch. 3).
 * ------------------------------------------------------------------- */
void oracle_dgemm_fp64(int64_t M, int64_t N, int64_t K, double alpha,
                       const double *A, int64_t lda, const double *B, int64_t ldb,
                       double beta, double *C, int64_t ldc)
{
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < M; ++i) {
            for (int64_t j = 0; j < N; ++j) acc[j] = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                double a = A[i * lda + k];
                const double *brow = B + k * ldb;
                for (int64_t j = 0; j < N; ++j) acc[j] = fma(a, brow[j], acc[j]);
            }
            for (int64_t j = 0; j < N; ++j) {
                double *c = C + i * ldc + j;
                *c = (beta == 0.0) ? alpha * acc[j] : fma(alpha, acc[j], beta * *c);
            }
        }
        free(acc);
    }
}

/* ---------------------------------------------------------------------
 * Double-double GEMM (error reference).  Per (i, j): s = 0; for each k the
 * exact product a*b = p + e (TwoProduct via fma) is added to s with the
 * accurate double-double addition (two TwoSums and two FastTwoSum
 * renormalisations; Dekker 1971, Knuth TAOCP 4.2.2, Hida-Li-Bailey QD).
 * ------------------------------------------------------------------- */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *s = x;
    *e = (a - av) + (b - bv);
}

static void fast_two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    *s = x;
    *e = b - (x - a);
}

static void dd_add(double ah, double al, double bh, double bl, double *rh, double *rl)
{
    double s1, s2, t1, t2;
    two_sum(ah, bh, &s1, &s2);
    two_sum(al, bl, &t1, &t2);
    s2 += t1;
    fast_two_sum(s1, s2, &s1, &s2);
    s2 += t2;
    fast_two_sum(s1, s2, rh, rl);
}

void oracle_dgemm_dd(int64_t M, int64_t N, int64_t K,
                     const double *A, int64_t lda, const double *B, int64_t ldb,
                     double *Chi, double *Clo, int64_t ldc)
{
#pragma omp parallel
    {
        double *hi = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
        double *lo = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < M; ++i) {
            for (int64_t j = 0; j < N; ++j) hi[j] = lo[j] = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                double a = A[i * lda + k];
                const double *brow = B + k * ldb;
                for (int64_t j = 0; j < N; ++j) {
                    double p = a * brow[j];
                    double e = fma(a, brow[j], -p);
                    dd_add(hi[j], lo[j], p, e, &hi[j], &lo[j]);
                }
            }
            for (int64_t j = 0; j < N; ++j) {
                Chi[i * ldc + j] = hi[j];
                Clo[i * ldc + j] = lo[j];
            }
        }
        free(hi);
        free(lo);
    }
}

/* ---------------------------------------------------------------------
 * Step 1 + 2: shared exponent and slices of one group (a row of A or a
 * column of B).
 * ------------------------------------------------------------------- */

/* Exponent shared by a group whose largest magnitude is mu. */
static int32_t shared_exponent(double mu)
{
    if (mu == 0.0) return 0;
    int E;
    double m = frexp(mu, &E); /* mu = m * 2^E, 0.5 <= m < 1 */
    return E + (m > 127.0 / 128.0 ? 1 : 0);
}

/* Balanced base-256 digits of X, most significant first: X = sum d[t] 256^(S-1-t). */
static void balanced_digits(int64_t X, int S, int8_t *d)
{
    for (int t = S - 1; t >= 1; --t) {
        int64_t r = X % 256; /* C remainder: same sign as X, |r| < 256 */
        if (r >= 128) r -= 256;
        if (r < -128) r += 256;
        d[t] = (int8_t)r;
        X = (X - r) / 256; /* exact */
    }
    d[0] = (int8_t)X;
}

/*
 * Split X (rows x cols, row-major, leading dimension ld) into S slices.
 * by_columns = 0: one exponent per row;  by_columns = 1: one per column.
 * digits: [S][rows][cols] (natural layout of X), exps: one per group,
 * bad: 1 for a group holding NaN or Inf (its digits are 0, exponent 0).
 * Returns the number of bad groups.
 */
int64_t oracle_split(int by_columns, int64_t rows, int64_t cols, const double *X, int64_t ld,
                     int S, int8_t *digits, int32_t *exps, uint8_t *bad)
{
    int64_t ngroups = by_columns ? cols : rows;
    int64_t len = by_columns ? rows : cols;
    int64_t nbad = 0;
#pragma omp parallel for schedule(static) reduction(+ : nbad)
    for (int64_t q = 0; q < ngroups; ++q) {
        double mu = 0.0;
        int nonfinite = 0;
        for (int64_t r = 0; r < len; ++r) {
            double x = by_columns ? X[r * ld + q] : X[q * ld + r];
            if (!isfinite(x)) nonfinite = 1;
            else if (fabs(x) > mu) mu = fabs(x);
        }
        int32_t e = nonfinite ? 0 : shared_exponent(mu);
        exps[q] = e;
        bad[q] = (uint8_t)nonfinite;
        nbad += nonfinite;
        for (int64_t r = 0; r < len; ++r) {
            double x = by_columns ? X[r * ld + q] : X[q * ld + r];
            int64_t fixed = nonfinite ? 0 : (int64_t)rint(ldexp(x, 8 * S - 1 - e));
            int8_t d[8];
            balanced_digits(fixed, S, d);
            int64_t i = by_columns ? r : q, j = by_columns ? q : r;
            for (int t = 0; t < S; ++t) digits[((int64_t)t * rows + i) * cols + j] = d[t];
        }
    }
    return nbad;
}

/* ---------------------------------------------------------------------
 * Step 3: every kept slice pair (s, t) multiplied exactly and added into
 * the accumulator of its diagonal g = s + t (kept when g < G).
 * Ad: [S][M][K] digits of A, Bd: [S][K][N] digits of B, Q: [G][M][N].
 * ------------------------------------------------------------------- */
void oracle_pair_products(int64_t M, int64_t N, int64_t K, int S, int G,
                          const int8_t *Ad, const int8_t *Bd, int64_t *Q)
{
    memset(Q, 0, sizeof(int64_t) * (size_t)G * (size_t)M * (size_t)N);
    for (int s = 0; s < S; ++s) {
        for (int t = 0; t < S; ++t) {
            int g = s + t;
            if (g >= G) continue;
            const int8_t *As = Ad + (int64_t)s * M * K;
            const int8_t *Bt = Bd + (int64_t)t * K * N;
            int64_t *Qg = Q + (int64_t)g * M * N;
            int64_t nblk = (N + 255) / 256;
#pragma omp parallel for collapse(2) schedule(static)
            for (int64_t i = 0; i < M; ++i) {
                for (int64_t jb = 0; jb < nblk; ++jb) {
                    int64_t j0 = jb * 256, j1 = j0 + 256 < N ? j0 + 256 : N;
                    int64_t *qrow = Qg + i * N;
                    for (int64_t k = 0; k < K; ++k) {
                        int64_t a = As[i * K + k];
                        const int8_t *brow = Bt + k * N;
                        for (int64_t j = j0; j < j1; ++j) qrow[j] += a * (int64_t)brow[j];
                    }
                }
            }
        }
    }
}

/* ---------------------------------------------------------------------
 * Step 4: Horner over the diagonals in FP64 from the least significant
 * one, then the shared scale 2^(e_i + f_j - 14), then alpha / beta.
 * ------------------------------------------------------------------- */
void oracle_recombine(int64_t M, int64_t N, int G, const int64_t *Q,
                      const int32_t *e, const int32_t *f,
                      const uint8_t *row_bad, const uint8_t *col_bad,
                      double alpha, double beta, double *C, int64_t ldc)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            double h = (double)Q[((int64_t)(G - 1) * M + i) * N + j];
            for (int g = G - 2; g >= 0; --g)
                h = h * 0x1p-8 + (double)Q[((int64_t)g * M + i) * N + j];
            double c = ldexp(h, e[i] + f[j] - 14);
            double *out = C + i * ldc + j;
            if (row_bad[i] || col_bad[j]) *out = NAN;
            else if (beta == 0.0) *out = alpha * c;
            else *out = fma(alpha, c, beta * *out);
        }
    }
}

/* ---------------------------------------------------------------------
 * The whole emulated GEMM: C = alpha * op(A) op(B) + beta * C with S slices
 * and G kept diagonals.  trans = 'N' or 'T' (BLAS meaning, row-major).
 * Returns 0, or -1 on bad arguments / allocation failure.
 * ------------------------------------------------------------------- */
int oracle_ozaki_dgemm(char transa, char transb, int64_t M, int64_t N, int64_t K,
                       double alpha, const double *A, int64_t lda,
                       const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                       int S, int G)
{
    if (S < 1 || S > 8 || G < 1 || G > 2 * S - 1 || M < 0 || N < 0 || K < 0) return -1;
    size_t mk = (size_t)M * (size_t)K, kn = (size_t)K * (size_t)N;
    double *opA = (double *)malloc(sizeof(double) * (mk ? mk : 1));
    double *opB = (double *)malloc(sizeof(double) * (kn ? kn : 1));
    int8_t *Ad = (int8_t *)malloc((size_t)S * (mk ? mk : 1));
    int8_t *Bd = (int8_t *)malloc((size_t)S * (kn ? kn : 1));
    int64_t *Q = (int64_t *)malloc(sizeof(int64_t) * (size_t)G * (size_t)(M * N > 0 ? M * N : 1));
    int32_t *e = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M ? M : 1));
    int32_t *f = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    uint8_t *rb = (uint8_t *)malloc((size_t)(M ? M : 1));
    uint8_t *cb = (uint8_t *)malloc((size_t)(N ? N : 1));
    int rc = 0;
    if (!opA || !opB || !Ad || !Bd || !Q || !e || !f || !rb || !cb) { rc = -1; goto done; }
    for (int64_t i = 0; i < M; ++i)
        for (int64_t k = 0; k < K; ++k)
            opA[i * K + k] = (transa == 'T' || transa == 't') ? A[k * lda + i] : A[i * lda + k];
    for (int64_t k = 0; k < K; ++k)
        for (int64_t j = 0; j < N; ++j)
            opB[k * N + j] = (transb == 'T' || transb == 't') ? B[j * ldb + k] : B[k * ldb + j];
    oracle_split(0, M, K, opA, K, S, Ad, e, rb);
    oracle_split(1, K, N, opB, N, S, Bd, f, cb);
    if (K == 0) {
        /* an empty row or column has exponent 0 and no digits */
        for (int64_t i = 0; i < M; ++i) { e[i] = 0; rb[i] = 0; }
        for (int64_t j = 0; j < N; ++j) { f[j] = 0; cb[j] = 0; }
    }
    oracle_pair_products(M, N, K, S, G, Ad, Bd, Q);
    oracle_recombine(M, N, G, Q, e, f, rb, cb, alpha, beta, C, ldc);
done:
    free(opA); free(opB); free(Ad); free(Bd); free(Q); free(e); free(f); free(rb); free(cb);
    return rc;
}
