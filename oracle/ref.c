/*
 * CPU oracle for the device data-sharing runtime -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct definitions of what one parallel region
 * computes once the master's implicitly shared locals have been handed to
 * the workers (paper: section 3.2, Figure 1b; section 5.1 "shared by
 * reference"; the Figure 5 and Figure 6 programs of section 6.1).  How the
 * locals are stored (team stack, LDS or HBM) does not change these results;
 * the stack behaviour itself is checked by the contention-group simulator
 * in sim.py.
 *
 * Only the tests, the package smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code with the GPU path.
 * Arithmetic is fp64 (the loop body fuses multiply-add with C99 fma(),
 * correctly rounded); integer work is exact.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Figure 1b pattern with four shared int32 scalars (a, b, c, d set by the
 * master before the parallel loop): iteration i of the worksharing loop
 * writes out[i] = a*i + b - (c XOR i) + d in 32-bit wrap-around arithmetic,
 * and adds out[i] into a shared 64-bit sum.  Fills out[0 .. hi-lo) for
 * i in [lo, hi) and returns the sum over that range. */
int64_t oref_affine_xor(int32_t a, int32_t b, int32_t c, int32_t d,
                        int64_t lo, int64_t hi, int32_t *out)
{
    int64_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) {
        uint32_t ui = (uint32_t)i;
        uint32_t v = (uint32_t)a * ui + (uint32_t)b - ((uint32_t)c ^ ui) + (uint32_t)d;
        int32_t o = (int32_t)v;
        if (out) out[i - lo] = o;
        sum += (int64_t)o;
    }
    return sum;
}

/* Scalar-sharing loop body (Figure 5 pattern generalised to K shared
 * scalars): y[i] = acc_K where acc_0 = arr[(i0+i) mod alen] as fp64 (or
 * +0.0 without a shared array) and each shared scalar s_k, int32 ones
 * first and fp64 ones after them, is applied as acc = fma(s_k, x[i], acc). */
void oref_fma_chain(const float *x, int64_t n,
                    const int32_t *si, int32_t ni,
                    const double *sf, int32_t nf,
                    const int32_t *arr, int64_t alen, int64_t i0,
                    double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double xi = (double)x[i];
        double acc = 0.0;
        if (alen > 0) acc = (double)arr[(i0 + i) % alen];
        for (int32_t k = 0; k < ni; ++k) acc = fma((double)si[k], xi, acc);
        for (int32_t k = 0; k < nf; ++k) acc = fma(sf[k], xi, acc);
        y[i] = acc;
    }
}

/* Array-sharing loop body (Figure 6 pattern with A shared arrays of one
 * length): out[i] = sum_j arr_j[i mod len] + i for i in [lo, hi).  arrs
 * holds the A arrays back to back. */
void oref_gather(const int32_t *arrs, int32_t A, int64_t len,
                 int64_t lo, int64_t hi, int32_t *out)
{
    for (int64_t i = lo; i < hi; ++i) {
        int64_t s = i;
        for (int32_t j = 0; j < A; ++j) s += arrs[(int64_t)j * len + (i % len)];
        out[i - lo] = (int32_t)(uint32_t)(uint64_t)s;
    }
}

/* ---- exact summation of doubles, rounded once to nearest-even ---------
 * The sum is held as one big signed integer in units of 2^-1074 (the
 * smallest subnormal), in 32-bit digits kept in int64 cells so that many
 * additions can be made before carries have to be propagated. */
#define OREF_DIGITS 72            /* 72*32 = 2304 bits > 2098 + headroom */

typedef struct { int64_t d[OREF_DIGITS]; int64_t pending; int status; } oref_acc;

static void acc_normalise(oref_acc *a)
{
    for (int k = 0; k < OREF_DIGITS - 1; ++k) {
        int64_t carry = a->d[k] >> 32;            /* floor division by 2^32 */
        a->d[k] -= carry * ((int64_t)1 << 32);
        a->d[k + 1] += carry;
    }
    a->pending = 0;
}

static void acc_add(oref_acc *a, double v)
{
    if (v == 0.0) return;
    if (!isfinite(v)) { a->status = 1; return; }
    uint64_t bits;
    memcpy(&bits, &v, 8);
    int neg = (int)(bits >> 63);
    int e = (int)((bits >> 52) & 0x7ff);
    uint64_t m = bits & ((1ull << 52) - 1);
    int shift;                                    /* v = m * 2^(shift-1074) */
    if (e == 0) shift = 0; else { m |= 1ull << 52; shift = e - 1; }
    int k = shift / 32, off = shift % 32;
    unsigned __int128 t = (unsigned __int128)m << off;
    int64_t p0 = (int64_t)(uint32_t)t;
    int64_t p1 = (int64_t)(uint32_t)(t >> 32);
    int64_t p2 = (int64_t)(uint32_t)(t >> 64);
    if (neg) { p0 = -p0; p1 = -p1; p2 = -p2; }
    a->d[k] += p0; a->d[k + 1] += p1; a->d[k + 2] += p2;
    if (++a->pending >= (1 << 20)) acc_normalise(a);
}

static double acc_round(oref_acc *a)
{
    if (a->status) return NAN;
    acc_normalise(a);
    int negative = a->d[OREF_DIGITS - 1] < 0;
    uint32_t mag[OREF_DIGITS];
    if (negative) {                               /* magnitude = -value */
        int64_t borrow = 0;
        for (int k = 0; k < OREF_DIGITS; ++k) {
            int64_t v = -a->d[k] - borrow;
            borrow = 0;
            while (v < 0) { v += (int64_t)1 << 32; borrow += 1; }
            mag[k] = (uint32_t)v;
        }
    } else {
        for (int k = 0; k < OREF_DIGITS; ++k) mag[k] = (uint32_t)a->d[k];
    }
    int top = -1;                                 /* highest set bit */
    for (int k = OREF_DIGITS - 1; k >= 0 && top < 0; --k)
        if (mag[k]) for (int b = 31; b >= 0; --b) if (mag[k] >> b & 1) { top = 32 * k + b; break; }
    if (top < 0) return 0.0;
#define BIT(p) ((p) >= 0 && (mag[(p) / 32] >> ((p) % 32) & 1u))
    double r;
    if (top <= 52) {                              /* fits 53 bits: exact */
        uint64_t m = 0;
        for (int p = top; p >= 0; --p) m = (m << 1) | BIT(p);
        r = ldexp((double)m, -1074);
    } else {
        uint64_t m = 0;
        for (int p = top; p > top - 53; --p) m = (m << 1) | BIT(p);
        int round = BIT(top - 53);
        int sticky = 0;
        for (int p = top - 54; p >= 0 && !sticky; --p) sticky = BIT(p);
        int lsb_pos = top - 52;                    /* weight of m's last bit */
        if (round && (sticky || (m & 1))) {
            m += 1;
            if (m == (1ull << 53)) { m >>= 1; lsb_pos += 1; }
        }
        r = ldexp((double)m, lsb_pos - 1074);      /* inf on overflow */
    }
#undef BIT
    return negative ? -r : r;
}

/* Correctly rounded (nearest, ties to even) value of the exact sum of
 * v[0..n).  status: 0 ok, 1 a non-finite input was seen (result NaN). */
double oref_exact_sum(const double *v, int64_t n, int32_t *status)
{
    oref_acc *a = (oref_acc *)calloc(1, sizeof(oref_acc));
    for (int64_t i = 0; i < n; ++i) acc_add(a, v[i]);
    double r = acc_round(a);
    if (status) *status = a->status;
    free(a);
    return r;
}

/* Exact sum of doubles v[0..n) that all lie on the 2^-75 grid, returned
 * as a signed 128-bit integer in units of 2^-75 (lo, hi words).  Returns
 * 0 if every value is on the grid and the total fits, 1 otherwise. */
int32_t oref_fixed75_sum(const double *v, int64_t n, uint64_t *lo, int64_t *hi)
{
    __int128 s = 0;
    for (int64_t i = 0; i < n; ++i) {
        double t = ldexp(v[i], 75);               /* exact scaling */
        if (!isfinite(t) || t != trunc(t) || fabs(t) >= 0x1p100) return 1;
        s += (__int128)t;
    }
    *lo = (uint64_t)s;
    *hi = (int64_t)(s >> 64);
    return 0;
}
