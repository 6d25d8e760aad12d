/*
 * Sanitizer run of the CPU oracle (test infrastructure): built with
 * -fsanitize=address,undefined together with oracle.c and run by
 * tests/test_sanitizers.py.  Every check has an exact expected value:
 *   - integer operands (|a|, |b| <= 2^20, S >= 5, G = S): the emulated GEMM
 *     equals the exact integer product (only digits t <= 2 are nonzero, so
 *     every kept pair is summed and every Horner partial sum is an integer
 *     below 2^53), also with transposes and alpha = 2, beta = -1 on an
 *     integer C;
 *   - digits reconstruct the fixed-point value RNE(x 2^(8S-1-e)) exactly and
 *     lie in the balanced ranges;
 *   - a NaN in a row of A gives a NaN row; K = 0 gives beta C;
 *   - the double-double GEMM of integer operands is exact;
 *   - out-of-range slice or diagonal counts are rejected.
 * Exits 0 when every check holds.
 */
#include "../../oracle/oracle.c"

#include <stdio.h>

static int failures = 0;
#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            fprintf(stderr, "FAIL: " __VA_ARGS__); \
            fprintf(stderr, "\n");                \
            ++failures;                           \
        }                                         \
    } while (0)

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64(void)
{
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
static int64_t rand_int(int64_t lim) { return (int64_t)(next_u64() % (uint64_t)(2 * lim + 1)) - lim; }
static double rand_unit(void) { return (double)(next_u64() >> 11) * 0x1p-53 * 2.0 - 1.0; }

static void integer_products(void)
{
    const int64_t M = 37, N = 29, K = 64;
    double *A = malloc(sizeof(double) * M * K), *B = malloc(sizeof(double) * K * N);
    double *AT = malloc(sizeof(double) * K * M), *BT = malloc(sizeof(double) * N * K);
    double *C = malloc(sizeof(double) * M * N), *C0 = malloc(sizeof(double) * M * N);
    int64_t *ref = malloc(sizeof(int64_t) * M * N);
    for (int64_t i = 0; i < M * K; ++i) A[i] = (double)rand_int(1 << 20);
    for (int64_t i = 0; i < K * N; ++i) B[i] = (double)rand_int(1 << 20);
    for (int64_t i = 0; i < M; ++i)
        for (int64_t k = 0; k < K; ++k) AT[k * M + i] = A[i * K + k];
    for (int64_t k = 0; k < K; ++k)
        for (int64_t j = 0; j < N; ++j) BT[j * K + k] = B[k * N + j];
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            int64_t s = 0;
            for (int64_t k = 0; k < K; ++k) s += (int64_t)A[i * K + k] * (int64_t)B[k * N + j];
            ref[i * N + j] = s;
            C0[i * N + j] = (double)rand_int(1000);
        }
    for (int S = 5; S <= 8; ++S) {
        CHECK(oracle_ozaki_dgemm('N', 'N', M, N, K, 1.0, A, K, B, N, 0.0, C, N, S, S) == 0, "dgemm S=%d", S);
        for (int64_t i = 0; i < M * N; ++i)
            CHECK(C[i] == (double)ref[i], "integer product S=%d elem %lld: %.17g vs %lld", S, (long long)i, C[i],
                  (long long)ref[i]);
        memcpy(C, C0, sizeof(double) * M * N);
        CHECK(oracle_ozaki_dgemm('T', 'T', M, N, K, 2.0, AT, M, BT, K, -1.0, C, N, S, S) == 0, "dgemm TT S=%d", S);
        for (int64_t i = 0; i < M * N; ++i)
            CHECK(C[i] == 2.0 * (double)ref[i] - C0[i], "alpha/beta S=%d elem %lld", S, (long long)i);
    }
    double *hi = malloc(sizeof(double) * M * N), *lo = malloc(sizeof(double) * M * N);
    oracle_dgemm_dd(M, N, K, A, K, B, N, hi, lo, N);
    for (int64_t i = 0; i < M * N; ++i) CHECK(hi[i] == (double)ref[i] && lo[i] == 0.0, "dd exact elem %lld", (long long)i);
    oracle_dgemm_fp64(M, N, K, 1.0, A, K, B, N, 0.0, C, N);
    for (int64_t i = 0; i < M * N; ++i) CHECK(C[i] == (double)ref[i], "fp64 exact elem %lld", (long long)i);
    free(A); free(B); free(AT); free(BT); free(C); free(C0); free(ref); free(hi); free(lo);
}

static void digits(void)
{
    const int64_t R = 9, L = 50;
    double *X = malloc(sizeof(double) * R * L);
    for (int64_t i = 0; i < R * L; ++i) X[i] = ldexp(rand_unit(), (int)rand_int(30));
    X[3 * L + 7] = 0.0;
    for (int64_t j = 0; j < L; ++j) X[5 * L + j] = 0.0; /* a zero row */
    for (int S = 2; S <= 8; ++S) {
        int8_t *d = malloc((size_t)S * R * L);
        int32_t e[9];
        uint8_t bad[9];
        CHECK(oracle_split(0, R, L, X, L, S, d, e, bad) == 0, "split S=%d", S);
        CHECK(e[5] == 0, "zero row exponent");
        for (int64_t i = 0; i < R; ++i)
            for (int64_t j = 0; j < L; ++j) {
                const int64_t want = (int64_t)rint(ldexp(X[i * L + j], 8 * S - 1 - e[i]));
                int64_t got = 0;
                for (int t = 0; t < S; ++t) {
                    const int v = d[((int64_t)t * R + i) * L + j];
                    got = got * 256 + v;
                    if (t == 0) CHECK(v >= -127 && v <= 127, "top digit range");
                }
                CHECK(got == want, "digits S=%d (%lld, %lld)", S, (long long)i, (long long)j);
            }
        free(d);
    }
    free(X);
}

static void special_cases(void)
{
    const int64_t M = 4, N = 3, K = 5;
    double A[20], B[15], C[12];
    for (int i = 0; i < 20; ++i) A[i] = rand_unit();
    for (int i = 0; i < 15; ++i) B[i] = rand_unit();
    A[1 * K + 2] = NAN;
    CHECK(oracle_ozaki_dgemm('N', 'N', M, N, K, 1.0, A, K, B, N, 0.0, C, N, 6, 6) == 0, "nan dgemm");
    for (int64_t j = 0; j < N; ++j) CHECK(isnan(C[1 * N + j]), "NaN row %lld", (long long)j);
    CHECK(!isnan(C[0]) && !isnan(C[2 * N]), "other rows finite");
    for (int i = 0; i < 12; ++i) C[i] = (double)i;
    CHECK(oracle_ozaki_dgemm('N', 'N', M, N, 0, 1.0, A, 1, B, N, 3.0, C, N, 6, 6) == 0, "K = 0");
    for (int i = 0; i < 12; ++i) CHECK(C[i] == 3.0 * i, "K = 0 gives beta C (%d)", i);
    CHECK(oracle_ozaki_dgemm('N', 'N', M, N, K, 1.0, A, K, B, N, 0.0, C, N, 9, 9) == -1, "S = 9 rejected");
    CHECK(oracle_ozaki_dgemm('N', 'N', M, N, K, 1.0, A, K, B, N, 0.0, C, N, 4, 8) == -1, "G = 2S rejected");
}

int main(void)
{
    integer_products();
    digits();
    special_cases();
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: all checks passed\n");
    return 0;
}
