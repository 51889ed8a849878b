/*
 * Sanitizer driver for oracle.c (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer together with oracle.c and
 * run on the CPU. It exercises every oracle entry point on small inputs whose
 * results are known in closed form (identity and integer products, rank-1
 * outer products, bfloat16 rounding of exact, tie and overflow values, the
 * splits) and on ragged leading dimensions, so that an out-of-bounds index or
 * undefined arithmetic in the oracle stops the run. Exit status 0: all checks
 * held and the sanitizers reported nothing.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_gemm_f64(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda,
                     const double *B, int64_t ldb, double *C, int64_t ldc);
void oracle_gemm_f64_omp(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda,
                         const double *B, int64_t ldb, double *C, int64_t ldc, int nthreads);
void oracle_gemm_entries_f64(int64_t k, const double *A, int64_t lda, const double *B,
                             int64_t ldb, const int64_t *rows, const int64_t *cols,
                             int64_t count, double *out);
uint16_t oracle_bf16_rne(float x);
void oracle_split_bf16(int64_t count, const float *x, uint16_t *hi, uint16_t *lo);
void oracle_split3_bf16(int64_t count, const float *x, uint16_t *hi, uint16_t *mid,
                        uint16_t *lo);
void oracle_bf16_rne_array(int64_t count, const float *x, uint16_t *out);
int oracle_max_threads(void);

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                  \
        }                                                                \
    } while (0)

static float bits_f(uint32_t u) { float f; memcpy(&f, &u, sizeof f); return f; }
static double bf16_value(uint16_t h) { return (double)bits_f((uint32_t)h << 16); }

int main(void)
{
    /* integer-valued product with padded leading dimensions, every order */
    enum { M = 7, K = 5, N = 6, LDA = 9, LDB = 8, LDC = 11 };
    double *A = malloc(sizeof(double) * M * LDA), *B = malloc(sizeof(double) * K * LDB);
    double *C = malloc(sizeof(double) * M * LDC), *C2 = malloc(sizeof(double) * M * LDC);
    for (int i = 0; i < M * LDA; ++i) A[i] = (double)((i * 7) % 17 - 8);
    for (int i = 0; i < K * LDB; ++i) B[i] = (double)((i * 5) % 17 - 8);
    oracle_gemm_f64(M, N, K, A, LDA, B, LDB, C, LDC);
    oracle_gemm_f64_omp(M, N, K, A, LDA, B, LDB, C2, LDC, 3);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int p = 0; p < K; ++p) s += A[i * LDA + p] * B[p * LDB + j];
            CHECK(C[i * LDC + j] == s);
            CHECK(C2[i * LDC + j] == s);
        }
    int64_t rows[4] = {0, 6, 3, 6}, cols[4] = {0, 5, 2, 0};
    double ent[4];
    oracle_gemm_entries_f64(K, A, LDA, B, LDB, rows, cols, 4, ent);
    for (int t = 0; t < 4; ++t) CHECK(ent[t] == C[rows[t] * LDC + cols[t]]);

    /* rank-1: (u v^T)(w z^T) = (v.w) u z^T, exact for small integers */
    double u[3] = {1, -2, 3}, v[4] = {2, 0, -1, 1}, w[4] = {1, 1, 2, -3}, z[2] = {4, -5};
    double R1[12], R2[8], R3[6];
    for (int i = 0; i < 3; ++i)
        for (int p = 0; p < 4; ++p) R1[i * 4 + p] = u[i] * v[p];
    for (int p = 0; p < 4; ++p)
        for (int j = 0; j < 2; ++j) R2[p * 2 + j] = w[p] * z[j];
    oracle_gemm_f64(3, 2, 4, R1, 4, R2, 2, R3, 2);
    const double vw = 2 * 1 + 0 * 1 + (-1) * 2 + 1 * (-3);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 2; ++j) CHECK(R3[i * 2 + j] == vw * u[i] * z[j]);

    /* k = 0 writes zeros; m = 0 or n = 0 writes nothing */
    double Z[4] = {5, 5, 5, 5};
    oracle_gemm_f64(2, 2, 0, A, 1, B, 2, Z, 2);
    for (int t = 0; t < 4; ++t) CHECK(Z[t] == 0.0);
    oracle_gemm_f64(0, 2, 3, NULL, 3, B, 2, NULL, 2);

    /* bfloat16 rounding: exact, tie to even (both directions), overflow */
    CHECK(oracle_bf16_rne(1.0f) == 0x3F80);
    CHECK(oracle_bf16_rne(bits_f(0x3F808000u)) == 0x3F80);   /* tie, even below */
    CHECK(oracle_bf16_rne(bits_f(0x3F818000u)) == 0x3F82);   /* tie, even above */
    CHECK(oracle_bf16_rne(bits_f(0x3F808001u)) == 0x3F81);
    CHECK(oracle_bf16_rne(bits_f(0x7F7FFFFFu)) == 0x7F80);   /* rounds to infinity */
    CHECK(oracle_bf16_rne(bits_f(0x00000001u)) == 0x0000);   /* smallest subnormal */
    CHECK(oracle_bf16_rne(-0.0f) == 0x8000);
    CHECK(isnan(bf16_value(oracle_bf16_rne(bits_f(0x7FC00001u)))));

    /* splits: hi + lo (+ mid) reproduce x exactly where the terms can */
    enum { S = 257 };
    float *x = malloc(sizeof(float) * S);
    uint16_t *hi = malloc(2 * S), *mid = malloc(2 * S), *lo = malloc(2 * S), *r = malloc(2 * S);
    for (int t = 0; t < S; ++t)
        x[t] = (float)((t * 2654435761u) % 100003) / 1000.0f - 50.0f;
    oracle_split_bf16(S, x, hi, lo);
    oracle_split3_bf16(S, x, r, mid, lo);
    oracle_bf16_rne_array(S, x, r);
    for (int t = 0; t < S; ++t) {
        CHECK(r[t] == hi[t]);
        const double s3 = bf16_value(hi[t]) + bf16_value(mid[t]) + bf16_value(lo[t]);
        CHECK(s3 == (double)x[t]);          /* 24 bits in three 8-bit terms */
    }
    CHECK(oracle_max_threads() >= 1);

    free(A); free(B); free(C); free(C2); free(x); free(hi); free(mid); free(lo); free(r);
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: all checks held\n");
    return 0;
}
