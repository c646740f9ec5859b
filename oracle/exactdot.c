/*
 * Correctly rounded dot products for the CPU oracle (test infrastructure).
 *
 * The coupling field of the coupled-oscillator model is a matrix-vector
 * product (paper, Sec. 3.1, Eq. (coup); Sec. 3.3 writes it as W^cp x).  The
 * paper notes that implementations differ in the order of their floating
 * point operations and that these differences grow along the trajectory
 * (Sec. 3.3, last paragraph).  The oracle removes that freedom by defining
 * each entry of the product as the exact real sum of the exact products,
 * rounded once to the nearest double (ties to even).
 *
 * Method: every double is an integer mantissa times a power of two, so each
 * product a*b is an integer of at most 106 bits times 2^(ea+eb).  Those
 * integers are added, exactly, into a fixed-point accumulator of signed
 * 64-bit limbs that each carry 32 bits of weight and 31 bits of headroom;
 * carries are resolved once at the end and the exact total is rounded to
 * nearest-even by inspecting its bits.  No floating point operation touches
 * the running sum, so the result does not depend on the order of terms.
 *
 * This file is compiled with gcc and loaded by the Python oracle; it shares
 * nothing with the HIP library.
 */
#include <stdint.h>
#include <string.h>
#include <math.h>

#define ACC_LOW_BIT (-2240)  /* accumulator bit 0 has weight 2^-2240        */
#define ACC_LIMBS   142      /* 142 * 32 = 4544 bits: weights up to 2^2303  */
#define ACC_FLUSH   (1 << 24) /* resolve carries at least this often        */

typedef struct {
    int64_t limb[ACC_LIMBS];
    int lo, hi;      /* range of limbs touched since the last reset */
    int64_t adds;    /* limb additions since the last carry resolution */
} acc_t;

static void acc_reset(acc_t *a)
{
    memset(a->limb, 0, sizeof a->limb);
    a->lo = ACC_LIMBS;
    a->hi = -1;
    a->adds = 0;
}

/* Split a finite double into sign, 53-bit integer mantissa and exponent:
 * v = sign * mant * 2^e. */
static void split_double(double v, int *sign, uint64_t *mant, int *e)
{
    uint64_t bits;
    memcpy(&bits, &v, sizeof bits);
    int be = (int)((bits >> 52) & 0x7ff);
    uint64_t f = bits & ((UINT64_C(1) << 52) - 1);
    *sign = (bits >> 63) ? -1 : 1;
    if (be == 0) {          /* zero or subnormal */
        *mant = f;
        *e = -1074;
    } else {
        *mant = f | (UINT64_C(1) << 52);
        *e = be - 1075;
    }
}

/* Resolve carries so that limbs 0..ACC_LIMBS-2 lie in [0, 2^32); the top
 * limb keeps the sign of the total. */
static void acc_carry(acc_t *a)
{
    for (int i = 0; i < ACC_LIMBS - 1; ++i) {
        int64_t c = a->limb[i] >> 32;          /* floor division by 2^32 */
        a->limb[i] -= c * (INT64_C(1) << 32);
        a->limb[i + 1] += c;
    }
    a->lo = 0;
    a->hi = ACC_LIMBS - 1;
    a->adds = 0;
}

/* Add sign * m * 2^pos exactly, where pos is the weight exponent of bit 0 of
 * m and m < 2^128. */
static void acc_add(acc_t *a, int sign, unsigned __int128 m, int pos)
{
    if (m == 0)
        return;
    int bit = pos - ACC_LOW_BIT;          /* >= 0 by construction */
    int li = bit >> 5;
    int sh = bit & 31;
    for (int j = 0; j < 4 && m != 0; ++j) {
        uint64_t chunk = (uint64_t)(m & 0xffffffffu);
        m >>= 32;
        if (chunk == 0)
            continue;
        uint64_t shifted = chunk << sh;   /* < 2^63 */
        int64_t lo = (int64_t)(shifted & 0xffffffffu);
        int64_t hi = (int64_t)(shifted >> 32);
        int k = li + j;
        if (sign > 0) {
            a->limb[k] += lo;
            a->limb[k + 1] += hi;
        } else {
            a->limb[k] -= lo;
            a->limb[k + 1] -= hi;
        }
        if (k < a->lo) a->lo = k;
        if (k + 1 > a->hi) a->hi = k + 1;
    }
    if (++a->adds >= ACC_FLUSH)
        acc_carry(a);
}

static int acc_bit(const acc_t *a, int i)
{
    return (int)((a->limb[i >> 5] >> (i & 31)) & 1);
}

/* Round the exact total to the nearest double, ties to even. */
static double acc_round(acc_t *a)
{
    acc_carry(a);
    int sign = 1;
    if (a->limb[ACC_LIMBS - 1] < 0) {
        sign = -1;
        for (int i = 0; i < ACC_LIMBS; ++i)
            a->limb[i] = -a->limb[i];
        acc_carry(a);
    }
    int top = -1;
    for (int i = ACC_LIMBS - 1; i >= 0; --i) {
        if (a->limb[i] != 0) {
            for (int b = 31; b >= 0; --b)
                if ((a->limb[i] >> b) & 1) { top = i * 32 + b; break; }
            break;
        }
    }
    if (top < 0)
        return 0.0;
    /* Bit index of the last place kept: 53 significant bits, but never below
     * the subnormal quantum 2^-1074. */
    int min_lsb = -1074 - ACC_LOW_BIT;
    int lsb = top - 52;
    if (lsb < min_lsb)
        lsb = min_lsb;
    uint64_t mant = 0;
    for (int i = top; i >= lsb; --i)
        mant = (mant << 1) | (uint64_t)acc_bit(a, i);
    int round_bit = (lsb - 1 >= 0) ? acc_bit(a, lsb - 1) : 0;
    int sticky = 0;
    for (int i = lsb - 2; i >= 0 && !sticky; --i)
        sticky = acc_bit(a, i);
    if (round_bit && (sticky || (mant & 1)))
        mant += 1;                       /* may carry to 2^53: still exact */
    double r = ldexp((double)mant, lsb + ACC_LOW_BIT);
    return sign > 0 ? r : -r;
}

static void acc_add_product(acc_t *acc, double x, double y)
{
    int sx, sy, ex, ey;
    uint64_t mx, my;
    split_double(x, &sx, &mx, &ex);
    split_double(y, &sy, &my, &ey);
    unsigned __int128 p = (unsigned __int128)mx * (unsigned __int128)my;
    acc_add(acc, sx * sy, p, ex + ey);
}

/* Nearest double to sum_{i<n} x[i*incx] * y[i*incy]; inputs must be finite. */
double exact_dot(const double *x, long incx, const double *y, long incy, long n)
{
    acc_t acc;
    acc_reset(&acc);
    for (long i = 0; i < n; ++i)
        acc_add_product(&acc, x[i * incx], y[i * incy]);
    return acc_round(&acc);
}

/* ------------------------------------------------------------------------
 * Certified fast path for the matrix-vector product.
 *
 * The superaccumulator above is the definition; it is also slow (tens of ns
 * per product).  For a row of the coupling product the nearest double to
 * the exact sum can usually be certified from a cheaper enclosure:
 *
 *  1. Error-free transformations (Ogita, Rump and Oishi, "Accurate sum and
 *     dot product", SIAM J. Sci. Comput. 26, 2005): TwoProduct gives
 *     x*y = h + r exactly (r = fma(x, y, -h)) when no underflow occurs, and
 *     Knuth's TwoSum gives p + h = p' + q exactly.  With LANES independent
 *     running sums and a final TwoSum of the lanes, the exact dot product
 *     is P + T, where P is a double and T the exact sum of every error term
 *     q and r.
 *  2. T is summed in floating point as S.  For m terms summed in any order
 *     |S - T| <= gamma_m sum|terms|, gamma_m = m u/(1 - m u), u = 2^-53
 *     (Higham, "Accuracy and Stability of Numerical Algorithms", Sec. 4.2).
 *     The sum of |terms| is itself summed in floating point as A; a bound
 *     E = 2 m u A covers both roundings while m u < 1e-3.
 *  3. TwoSum(P, S) = (hi, lo) exactly, so the exact result X lies in
 *     [hi + lo - E, hi + lo + E].  hi is the nearest double to X if that
 *     interval lies strictly inside (hi - g/2, hi + g/2), where g is the
 *     smaller of the two gaps from hi to its neighbouring doubles.
 *
 * Any row that fails the test (a result too close to a rounding boundary,
 * a zero or subnormal result, a product outside [2^-960, 2^960] in
 * magnitude where TwoProduct might not be exact, non-finite data) is
 * recomputed with the superaccumulator.  The result is therefore the
 * nearest double to the exact sum for every row, whichever path produced it.
 * ---------------------------------------------------------------------- */
#include <omp.h>

#define LANES 8
#define EXACT_PARALLEL_MIN (1L << 16)

static long g_fallbacks = 0;    /* rows sent to the superaccumulator */

/* One row: returns 1 and sets *res when certified, 0 otherwise. */
#define FAST_ROW_BODY                                                          \
    double P[LANES], Eacc[LANES], Aacc[LANES];                                 \
    int bad[LANES];                                                            \
    for (int j = 0; j < LANES; ++j) {                                          \
        P[j] = 0.0; Eacc[j] = 0.0; Aacc[j] = 0.0; bad[j] = 0;                  \
    }                                                                          \
    long i = 0;                                                                \
    for (; i + LANES <= n; i += LANES) {                                       \
        _Pragma("omp simd")                                                    \
        for (int j = 0; j < LANES; ++j) {                                      \
            double a = x[i + j], b = y[i + j];                                 \
            double h = a * b;                                                  \
            double r = fma(a, b, -h);                                          \
            double p = P[j];                                                   \
            double s = p + h;                                                  \
            double bb = s - p;                                                 \
            double q = (p - (s - bb)) + (h - bb);                              \
            P[j] = s;                                                          \
            Eacc[j] += q + r;                                                  \
            Aacc[j] += fabs(q) + fabs(r);                                      \
            double ah = fabs(h);                                               \
            bad[j] |= ((ah < 0x1p-960) & (a != 0.0) & (b != 0.0))              \
                      | !(ah <= 0x1p960);                                      \
        }                                                                      \
    }                                                                          \
    for (; i < n; ++i) {                                                       \
        double a = x[i], b = y[i];                                             \
        double h = a * b;                                                      \
        double r = fma(a, b, -h);                                              \
        double p = P[0];                                                       \
        double s = p + h;                                                      \
        double bb = s - p;                                                     \
        double q = (p - (s - bb)) + (h - bb);                                  \
        P[0] = s;                                                              \
        Eacc[0] += q + r;                                                      \
        Aacc[0] += fabs(q) + fabs(r);                                          \
        double ah = fabs(h);                                                   \
        bad[0] |= ((ah < 0x1p-960) & (a != 0.0) & (b != 0.0))                  \
                  | !(ah <= 0x1p960);                                          \
    }                                                                          \
    double Pt = P[0], St = Eacc[0], At = Aacc[0];                              \
    int anybad = bad[0];                                                       \
    for (int j = 1; j < LANES; ++j) {                                          \
        double s = Pt + P[j];                                                  \
        double bb = s - Pt;                                                    \
        double q = (Pt - (s - bb)) + (P[j] - bb);                              \
        Pt = s;                                                                \
        St += q + Eacc[j];                                                     \
        At += fabs(q) + Aacc[j];                                               \
        anybad |= bad[j];                                                      \
    }                                                                          \
    double hi = Pt + St;                                                       \
    double bb = hi - Pt;                                                       \
    double lo = (Pt - (hi - bb)) + (St - bb);                                  \
    double m_terms = 2.0 * (double)n + 4.0 * LANES;                            \
    double E = 2.0 * m_terms * 0x1p-53 * At;                                   \
    if (anybad || !(hi != 0.0) || !isfinite(hi) || !isfinite(E)                \
        || fabs(hi) < 0x1p-1000 || m_terms * 0x1p-53 >= 1e-3)                  \
        return 0;                                                              \
    double gu = nextafter(hi, INFINITY) - hi;                                  \
    double gd = hi - nextafter(hi, -INFINITY);                                 \
    double g = gu < gd ? gu : gd;                                              \
    if (!((fabs(lo) + E) * (1.0 + 0x1p-40) < 0.5 * g))                         \
        return 0;                                                              \
    *res = hi;                                                                 \
    return 1;

__attribute__((target("avx2,fma")))
static int fast_dot_avx2(const double *x, const double *y, long n, double *res)
{
    FAST_ROW_BODY
}

static int fast_dot_generic(const double *x, const double *y, long n, double *res)
{
    FAST_ROW_BODY
}

/* out[k] = nearest double to sum_i A[k*lda + i] * x[i], for k < rows, by the
 * superaccumulator alone.  Rows are independent, so they may be evaluated
 * by several threads without changing any result. */
void exact_matvec_reference(const double *A, long rows, long cols, long lda,
                            const double *x, double *out)
{
#pragma omp parallel for schedule(static) if (rows * cols >= EXACT_PARALLEL_MIN)
    for (long k = 0; k < rows; ++k)
        out[k] = exact_dot(A + k * lda, 1, x, 1, cols);
}

/* out[k] = nearest double to sum_i A[k*lda + i] * x[i], for k < rows: the
 * certified fast path where it decides, the superaccumulator elsewhere.
 * The result equals exact_matvec_reference bit for bit. */
void exact_matvec(const double *A, long rows, long cols, long lda,
                  const double *x, double *out)
{
    int (*fast)(const double *, const double *, long, double *) =
        (__builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma"))
            ? fast_dot_avx2 : fast_dot_generic;
    long fb = 0;
    /* small products stay on one thread: a parallel region costs more than
     * they do (the rows are independent either way) */
#pragma omp parallel for schedule(static) reduction(+:fb) if (rows * cols >= EXACT_PARALLEL_MIN)
    for (long k = 0; k < rows; ++k) {
        double v;
        if (!fast(A + k * lda, x, cols, &v)) {
            v = exact_dot(A + k * lda, 1, x, 1, cols);
            ++fb;
        }
        out[k] = v;
    }
#pragma omp atomic
    g_fallbacks += fb;
}

/* Rows exact_matvec has sent to the superaccumulator since the library was
 * loaded (a test hook: shows which path decided). */
long exact_fallbacks(void) { return g_fallbacks; }

/* Exact sum of n doubles, rounded once (the sum of x[i] * 1.0). */
double exact_sum(const double *x, long n)
{
    acc_t acc;
    acc_reset(&acc);
    for (long i = 0; i < n; ++i)
        acc_add_product(&acc, x[i], 1.0);
    return acc_round(&acc);
}

/* Number of threads exact_matvec uses (OpenMP's current maximum). */
int exact_threads(void) { return omp_get_max_threads(); }
