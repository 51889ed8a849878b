/*
 * Plain CPU oracle for the dense product C = A*B.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it. It shares no code, header or constant with
 * the HIP path.
 *
 * Source: D.T. Hasta and A.B. Mutiara, "Performance Evaluation of Parallel
 * Message Passing and Thread Programming Model on Multicore Architectures"
 * (arXiv 1012.2273).
 *   - Section 3.1, Algorithm 1: the sequential product, loop nest
 *     (row, column, reduction) with the reduction innermost.
 *   - Section 3.1.1, Algorithm 3 and Section 3.1.2, Algorithm 4: every
 *     c[i][k] is set to zero before its reduction, so C is overwritten.
 *   - Section 3.1.2, Algorithm 4: the same loop nest with the row loop
 *     shared among threads by "omp for" (used here only to time the paper's
 *     multicore baseline and to check large sizes faster; it yields the same
 *     bits because each entry is still summed in ascending reduction order).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * No fused multiply-add: every product and every sum is rounded separately,
 * so the serial, threaded and sampled-entry routines agree bit for bit.
 */
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <omp.h>

/* C(m x n) = A(m x k) * B(k x n); row-major with leading dimensions in
 * elements. Section 3.1, Algorithm 1 (loop order) with the zeroing of
 * Algorithms 3 and 4. */
void oracle_gemm_f64(int64_t m, int64_t n, int64_t k,
                     const double *A, int64_t lda,
                     const double *B, int64_t ldb,
                     double *C, int64_t ldc)
{
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int64_t p = 0; p < k; ++p) {
                double prod = A[i * lda + p] * B[p * ldb + j];
                s = s + prod;
            }
            C[i * ldc + j] = s;
        }
    }
}

/* Section 3.1.2, Algorithm 4: the row loop is divided among `nthreads`
 * threads with a static schedule; the per-entry arithmetic is unchanged. */
void oracle_gemm_f64_omp(int64_t m, int64_t n, int64_t k,
                         const double *A, int64_t lda,
                         const double *B, int64_t ldb,
                         double *C, int64_t ldc, int nthreads)
{
    int64_t i;
#pragma omp parallel for schedule(static) num_threads(nthreads) private(i)
    for (i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int64_t p = 0; p < k; ++p) {
                double prod = A[i * lda + p] * B[p * ldb + j];
                s = s + prod;
            }
            C[i * ldc + j] = s;
        }
    }
}

/* Selected entries of the same product: out[t] = C[rows[t]][cols[t]], each
 * summed exactly as above. Used where the full product is too slow on the
 * CPU; the values are bit-identical to the full routines. */
void oracle_gemm_entries_f64(int64_t k,
                             const double *A, int64_t lda,
                             const double *B, int64_t ldb,
                             const int64_t *rows, const int64_t *cols,
                             int64_t count, double *out)
{
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = rows[t], j = cols[t];
        double s = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            double prod = A[i * lda + p] * B[p * ldb + j];
            s = s + prod;
        }
        out[t] = s;
    }
}

/*
 * Round a binary32 value to the nearest bfloat16 (8-bit significand),
 * ties to even, written from the IEEE 754 definition: the two bfloat16
 * values that bracket x are the one obtained by cutting the low 16 bits
 * (toward zero) and its neighbour away from zero; pick the nearer, and on a
 * tie the one whose last kept bit is 0. NaN stays NaN (quiet), infinities
 * and zeros are exact. Returns the 16-bit pattern.
 */
uint16_t oracle_bf16_rne(float x)
{
    uint32_t u;
    memcpy(&u, &x, sizeof u);
    if (isnan(x))
        return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t lo_bits = u & 0xFFFF0000u;          /* toward zero          */
    if ((u & 0x0000FFFFu) == 0)
        return (uint16_t)(lo_bits >> 16);        /* already representable */
    uint32_t hi_bits = lo_bits + 0x00010000u;    /* away from zero        */
    float below, above;
    memcpy(&below, &lo_bits, sizeof below);
    memcpy(&above, &hi_bits, sizeof above);
    /* distances computed exactly in binary64 (all three are binary32) */
    double d_below = fabs((double)x - (double)below);
    double d_above = isinf(above) ? INFINITY : fabs((double)above - (double)x);
    if (isinf(above)) {
        /* the neighbour past the largest finite bfloat16 is infinity; it is
         * chosen when x is at or beyond the midpoint, where the midpoint is
         * the largest finite value plus half its last-place unit */
        double maxfin = fabs((double)below);
        double half_ulp = ldexp(1.0, ilogb(maxfin) - 8);
        double mag = fabs((double)x);
        if (mag >= maxfin + half_ulp)
            return (uint16_t)(hi_bits >> 16);
        return (uint16_t)(lo_bits >> 16);
    }
    if (d_below < d_above)
        return (uint16_t)(lo_bits >> 16);
    if (d_above < d_below)
        return (uint16_t)(hi_bits >> 16);
    /* tie: keep the candidate with an even last bit */
    return ((lo_bits >> 16) & 1u) ? (uint16_t)(hi_bits >> 16)
                                  : (uint16_t)(lo_bits >> 16);
}

static float bf16_bits_to_float(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return f;
}

/*
 * Two-term bfloat16 split of binary32 data: hi = bf16(x), lo = bf16(x - hi).
 * The difference x - hi is computed in binary64, where it is exact, and it is
 * also exactly representable in binary32 (it is x with its top 8 significand
 * bits removed), so the narrowing cast below is exact.
 */
void oracle_split_bf16(int64_t count, const float *x, uint16_t *hi, uint16_t *lo)
{
    for (int64_t t = 0; t < count; ++t) {
        uint16_t h = oracle_bf16_rne(x[t]);
        double r = (double)x[t] - (double)bf16_bits_to_float(h);
        hi[t] = h;
        lo[t] = oracle_bf16_rne((float)r);
    }
}

/*
 * Three-term bfloat16 split of binary32 data: hi = bf16(x), mid = bf16(x - hi),
 * lo = bf16(x - hi - mid). Each difference is computed in binary64, where it
 * is exact; it is also exactly representable in binary32 (x with its leading
 * significand bits removed: the second difference is of two binary32 values
 * within a factor two of each other), so the narrowing casts are exact.
 */
void oracle_split3_bf16(int64_t count, const float *x, uint16_t *hi, uint16_t *mid,
                        uint16_t *lo)
{
    for (int64_t t = 0; t < count; ++t) {
        uint16_t h = oracle_bf16_rne(x[t]);
        double r1 = (double)x[t] - (double)bf16_bits_to_float(h);
        uint16_t m = oracle_bf16_rne((float)r1);
        double r2 = r1 - (double)bf16_bits_to_float(m);
        hi[t] = h;
        mid[t] = m;
        lo[t] = oracle_bf16_rne((float)r2);
    }
}

/* Batch form of oracle_bf16_rne. */
void oracle_bf16_rne_array(int64_t count, const float *x, uint16_t *out)
{
    for (int64_t t = 0; t < count; ++t)
        out[t] = oracle_bf16_rne(x[t]);
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
