/*
 * Host driver for the oracle's exact dot product under AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure; built and run by
 * tests/test_oracle_sanitizers.py).  It exercises every branch of the
 * superaccumulator and of the certified fast path -- subnormal, huge and
 * cancelling products, strided access, rows long enough to force the
 * periodic carry resolution -- and checks that the fast path equals the
 * superaccumulator bit for bit and that sums with an integer closed form
 * come out exact.  Exit status 0 and a final "ok" line on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double exact_dot(const double *x, long incx, const double *y, long incy, long n);
void exact_matvec_reference(const double *A, long rows, long cols, long lda, const double *x, double *out);
void exact_matvec(const double *A, long rows, long cols, long lda, const double *x, double *out);
double exact_sum(const double *x, long n);

static uint64_t state = 0x9e3779b97f4a7c15ULL;

static uint64_t next(void)   /* splitmix64 */
{
    uint64_t z = (state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static double uniform(void) { return (double)(next() >> 11) * 0x1p-53; }

/* a finite double of random sign with exponent in [lo, hi] (subnormals included) */
static double wide(int lo, int hi)
{
    double m = 1.0 + uniform();
    int e = lo + (int)(next() % (uint64_t)(hi - lo + 1));
    double v = ldexp(m, e);
    return (next() & 1) ? -v : v;
}

static int same_bits(double a, double b)
{
    uint64_t x, y;
    memcpy(&x, &a, 8);
    memcpy(&y, &b, 8);
    return x == y;
}

static int failures = 0;

static void check(int ok, const char *what, long i)
{
    if (!ok) {
        fprintf(stderr, "FAIL %s (row %ld)\n", what, i);
        ++failures;
    }
}

/* rows x cols matrix in one of several regimes; fast path vs reference */
static void regime(const char *name, long rows, long cols, int lo, int hi, int cancel)
{
    const long lda = cols + 3;
    double *A = malloc(sizeof(double) * rows * lda), *x = malloc(sizeof(double) * cols);
    double *r1 = malloc(sizeof(double) * rows), *r2 = malloc(sizeof(double) * rows);
    for (long j = 0; j < cols; ++j) x[j] = wide(lo, hi);
    for (long k = 0; k < rows; ++k)
        for (long j = 0; j < lda; ++j) A[k * lda + j] = wide(lo, hi);
    if (cancel)   /* second half of each row cancels the first: tiny results */
        for (long k = 0; k < rows; ++k)
            for (long j = 0; j + 1 < cols; j += 2) {
                A[k * lda + j + 1] = -A[k * lda + j] * (1.0 + 0x1p-50 * (double)(k % 5));
                x[j + 1] = x[j];
            }
    exact_matvec(A, rows, cols, lda, x, r1);
    exact_matvec_reference(A, rows, cols, lda, x, r2);
    for (long k = 0; k < rows; ++k) check(same_bits(r1[k], r2[k]), name, k);
    /* strided access: column 0 of A against x read backwards through a stride of 2 */
    double *xs = malloc(sizeof(double) * 2 * cols), *col = malloc(sizeof(double) * cols);
    for (long j = 0; j < cols; ++j) {
        xs[2 * j] = x[j];
        xs[2 * j + 1] = NAN;   /* never read */
    }
    long n = rows < cols ? rows : cols;
    for (long j = 0; j < n; ++j) col[j] = A[j * lda];
    check(same_bits(exact_dot(A, lda, xs, 2, n), exact_dot(col, 1, x, 1, n)), name, -1);
    free(A); free(x); free(r1); free(r2); free(xs); free(col);
}

int main(void)
{
    regime("ordinary", 64, 1000, -4, 4, 0);
    regime("wide exponents", 64, 257, -300, 300, 0);
    regime("subnormal products", 32, 129, -1074, -500, 0);
    regime("huge products", 32, 129, 400, 1000, 0);
    regime("cancelling", 64, 512, -10, 10, 1);
    regime("tail only", 16, 7, -3, 3, 0);
    regime("empty rows", 4, 0, 0, 0, 0);

    /* closed forms: integer terms times a power of two are exact as long as
     * the integer total fits 53 bits; 4M terms force the periodic carry
     * resolution of the accumulator */
    const long big = 4L << 20;
    double *a = malloc(sizeof(double) * big), *b = malloc(sizeof(double) * big);
    int64_t total = 0;
    for (long i = 0; i < big; ++i) {
        int64_t k = (int64_t)(next() % (1u << 20)) - (1 << 19);
        a[i] = (double)k;
        b[i] = 0x1p-30;
        total += k;
    }
    check(same_bits(exact_dot(a, 1, b, 1, big), ldexp((double)total, -30)), "integer closed form", big);
    check(same_bits(exact_sum(a, big), (double)total), "exact_sum closed form", big);
    /* ties to even: 1 + 2^-53 rounds to 1, 1 + 3*2^-53 rounds up to 1 + 2^-51 */
    double t1[3] = {1.0, 0x1p-53, 0.0}, t2[3] = {1.0, 0x1p-53, 0x1p-52};
    check(same_bits(exact_sum(t1, 3), 1.0), "tie to even (down)", 0);
    check(same_bits(exact_sum(t2, 3), 1.0 + 0x1p-51), "tie to even (up)", 0);
    /* total cancellation of huge terms leaves the tiny one exactly */
    double t3[4] = {0x1p1000, 0x1p-1074, -0x1p1000, 0.0};
    check(same_bits(exact_sum(t3, 4), 0x1p-1074), "cancellation to the smallest subnormal", 0);
    free(a);
    free(b);
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
