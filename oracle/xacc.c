/*
 * xacc.c: exact fixed-point accumulator (test infrastructure, see
 * twofold_oracle.h).
 *
 * Defines the exact target of the paper's twofold results: S = sum x_n or
 * S = sum x_n*y_n ("Overview": value + error approximates an exact real).
 * Every binary64 number is an integer m < 2^53 times 2^e with
 * e >= -1074, so every product of two binary64 numbers is an integer
 * m1*m2 < 2^106 times 2^(e1+e2) with e1+e2 >= -2148. The accumulator is a
 * long fixed-point integer whose bit 0 weighs 2^XACC_LSB (XACC_LSB = -2272,
 * below every such weight) and whose top reaches 2^2272, far above any
 * finite sum of products of binary64 numbers. Adding is exact integer
 * addition; binary32 inputs are first widened to binary64, which is exact.
 *
 * Representation: XACC_NDIG signed 64-bit "digits" of base 2^32. An add
 * spreads the (shifted) mantissa over up to five digits without carrying,
 * each digit changing by less than 2^33; carries are propagated every
 * XACC_RENORM adds and before rounding, so no digit ever overflows.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "twofold_oracle.h"

#define XACC_NDIG 142
#define XACC_LSB (-2272)
#define XACC_RENORM (1 << 26)

typedef struct {
  int64_t dig[XACC_NDIG]; /* value = sum dig[i] * 2^(32*i + XACC_LSB) */
  int64_t nadd;           /* adds since the last carry propagation      */
  int nan, pinf, ninf;    /* non-finite terms seen                      */
} xacc_t;

size_t oracle_xacc_size(void) { return sizeof(xacc_t); }

void oracle_xacc_clear(void* acc) { memset(acc, 0, sizeof(xacc_t)); }

/* Propagate carries so that dig[0..NDIG-2] lie in [0, 2^32) and the top
 * digit carries the sign. gcc's >> on a negative int64 is an arithmetic
 * shift, i.e. floor division by 2^32. */
static void xacc_carry(xacc_t* a) {
  for (int i = 0; i < XACC_NDIG - 1; i++) {
    int64_t c = a->dig[i] >> 32;
    a->dig[i] -= c * (int64_t)4294967296LL;
    a->dig[i + 1] += c;
  }
  a->nadd = 0;
}

/* Add (or subtract, when neg) the integer m times 2^e. Requires
 * e >= XACC_LSB and m < 2^128. */
static void xacc_add_int(xacc_t* a, unsigned __int128 m, int e, int neg) {
  if (m == 0) return;
  int pos = e - XACC_LSB;
  int idx = pos >> 5, sh = pos & 31;
  for (int k = 0; k < 4; k++) {
    uint64_t chunk = (uint64_t)(m >> (32 * k)) & 0xFFFFFFFFull;
    if (chunk == 0) continue;
    uint64_t v = chunk << sh; /* < 2^63 */
    int64_t lo = (int64_t)(v & 0xFFFFFFFFull), hi = (int64_t)(v >> 32);
    if (neg) {
      a->dig[idx + k] -= lo;
      a->dig[idx + k + 1] -= hi;
    } else {
      a->dig[idx + k] += lo;
      a->dig[idx + k + 1] += hi;
    }
  }
  if (++a->nadd >= XACC_RENORM) xacc_carry(a);
}

/* Record a non-finite term; returns 1 if x is not finite. */
static int xacc_nonfinite(xacc_t* a, double x) {
  if (isnan(x)) { a->nan = 1; return 1; }
  if (isinf(x)) { if (x > 0) a->pinf = 1; else a->ninf = 1; return 1; }
  return 0;
}

/* x = (-1)^neg * m * 2^e with m an integer below 2^53 (exact for any
 * finite binary64, subnormals included: frexp normalises them). */
static void split_f64(double x, uint64_t* m, int* e, int* neg) {
  int ex;
  double f = frexp(fabs(x), &ex); /* |x| = f * 2^ex, f in [0.5, 1) */
  *m = (uint64_t)ldexp(f, 53);
  *e = ex - 53;
  *neg = signbit(x) ? 1 : 0;
}

static void xacc_add_f64(xacc_t* a, double x, int absval) {
  if (xacc_nonfinite(a, absval ? fabs(x) : x)) return;
  if (x == 0) return;
  uint64_t m;
  int e, neg;
  split_f64(x, &m, &e, &neg);
  xacc_add_int(a, m, e, absval ? 0 : neg);
}

static void xacc_add_prod_f64(xacc_t* a, double x, double y, int absval) {
  if (!isfinite(x) || !isfinite(y)) {
    /* IEEE product of the non-finite operands (0*inf gives NaN). */
    double p = x * y;
    xacc_nonfinite(a, absval ? fabs(p) : p);
    return;
  }
  if (x == 0 || y == 0) return;
  uint64_t mx, my;
  int ex, ey, nx, ny;
  split_f64(x, &mx, &ex, &nx);
  split_f64(y, &my, &ey, &ny);
  unsigned __int128 m = (unsigned __int128)mx * my;
  xacc_add_int(a, m, ex + ey, absval ? 0 : (nx ^ ny));
}

static void xacc_merge(xacc_t* dst, const xacc_t* src) {
  xacc_t s = *src;
  xacc_carry(&s);
  xacc_carry(dst);
  for (int i = 0; i < XACC_NDIG; i++) dst->dig[i] += s.dig[i];
  xacc_carry(dst);
  dst->nan |= src->nan;
  dst->pinf |= src->pinf;
  dst->ninf |= src->ninf;
}

/* ---- threaded range adds ---------------------------------------------- */

typedef struct {
  xacc_t acc;
  int kind; /* 0 sum f32, 1 sum f64, 2 dot f32, 3 dot f64 */
  const void *x, *y;
  int64_t lo, hi;
  int absval;
} slice_t;

static void* slice_run(void* arg) {
  slice_t* s = (slice_t*)arg;
  for (int64_t i = s->lo; i < s->hi; i++) {
    switch (s->kind) {
      case 0: xacc_add_f64(&s->acc, (double)((const float*)s->x)[i], s->absval); break;
      case 1: xacc_add_f64(&s->acc, ((const double*)s->x)[i], s->absval); break;
      case 2:
        xacc_add_prod_f64(&s->acc, (double)((const float*)s->x)[i],
                          (double)((const float*)s->y)[i], s->absval);
        break;
      default:
        xacc_add_prod_f64(&s->acc, ((const double*)s->x)[i], ((const double*)s->y)[i],
                          s->absval);
        break;
    }
  }
  return NULL;
}

static void add_range(void* acc, int kind, const void* x, const void* y, int64_t n, int absval,
                      int nthreads) {
  if (n <= 0) return;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((int64_t)nthreads > n) nthreads = (int)n;
  slice_t* sl = (slice_t*)calloc((size_t)nthreads, sizeof(slice_t));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  int* started = (int*)calloc((size_t)nthreads, sizeof(int));
  for (int t = 0; t < nthreads; t++) {
    sl[t].kind = kind;
    sl[t].x = x;
    sl[t].y = y;
    sl[t].lo = n * t / nthreads;
    sl[t].hi = n * (t + 1) / nthreads;
    sl[t].absval = absval;
    if (t > 0 && pthread_create(&th[t], NULL, slice_run, &sl[t]) == 0) started[t] = 1;
  }
  slice_run(&sl[0]);
  for (int t = 1; t < nthreads; t++) {
    if (started[t])
      pthread_join(th[t], NULL);
    else
      slice_run(&sl[t]); /* thread creation failed: do the slice here */
  }
  for (int t = 0; t < nthreads; t++) xacc_merge((xacc_t*)acc, &sl[t].acc);
  free(sl);
  free(th);
  free(started);
}

void oracle_xacc_add_sum_f32(void* acc, const float* x, int64_t n, int abs_values, int nthreads) {
  add_range(acc, 0, x, NULL, n, abs_values, nthreads);
}
void oracle_xacc_add_sum_f64(void* acc, const double* x, int64_t n, int abs_values, int nthreads) {
  add_range(acc, 1, x, NULL, n, abs_values, nthreads);
}
void oracle_xacc_add_dot_f32(void* acc, const float* x, const float* y, int64_t n, int abs_values,
                             int nthreads) {
  add_range(acc, 2, x, y, n, abs_values, nthreads);
}
void oracle_xacc_add_dot_f64(void* acc, const double* x, const double* y, int64_t n,
                             int abs_values, int nthreads) {
  add_range(acc, 3, x, y, n, abs_values, nthreads);
}

/* ---- rounding ------------------------------------------------------------ */

static int bit_at(const xacc_t* a, int i) { return (int)((a->dig[i >> 5] >> (i & 31)) & 1); }

/* Sign and magnitude: on return *mag holds |value| with every digit in
 * [0, 2^32); returns 1 if the value is negative. */
static int xacc_magnitude(const xacc_t* src, xacc_t* mag) {
  *mag = *src;
  xacc_carry(mag);
  int neg = mag->dig[XACC_NDIG - 1] < 0;
  if (neg) {
    for (int i = 0; i < XACC_NDIG; i++) mag->dig[i] = -mag->dig[i];
    xacc_carry(mag);
  }
  return neg;
}

static double round_value(const xacc_t* src, int prec, int emin_sub) {
  if (src->nan || (src->pinf && src->ninf)) return NAN;
  if (src->pinf) return INFINITY;
  if (src->ninf) return -INFINITY;
  xacc_t m;
  int neg = xacc_magnitude(src, &m);
  int nbits = 32 * XACC_NDIG;
  int hb = -1;
  for (int i = nbits - 1; i >= 0; i--)
    if (bit_at(&m, i)) { hb = i; break; }
  if (hb < 0) return 0.0;
  /* Bit index of the unit in the last place: prec bits below and including
   * hb, but never below the smallest subnormal's weight. */
  int q = hb - (prec - 1);
  int qmin = emin_sub - XACC_LSB;
  if (q < qmin) q = qmin;
  uint64_t mant = 0;
  for (int i = hb; i >= q; i--) mant = (mant << 1) | (uint64_t)bit_at(&m, i);
  int rnd = (q >= 1) ? bit_at(&m, q - 1) : 0;
  int sticky = 0;
  for (int i = q - 2; i >= 0 && !sticky; i--) sticky = bit_at(&m, i);
  if (rnd && (sticky || (mant & 1))) mant++;
  /* mant <= 2^prec, exactly representable in binary64 for prec <= 53;
   * ldexp is exact here and overflows to infinity as RN requires. The
   * binary32 case returns a binary64 holding the binary32 value, so
   * prec 24 results above the binary32 range must be checked by callers. */
  double r = ldexp((double)mant, q + XACC_LSB);
  return neg ? -r : r;
}

double oracle_xacc_round(const void* acc, int prec_bits, int emin_sub) {
  return round_value((const xacc_t*)acc, prec_bits, emin_sub);
}

double oracle_xacc_round_diff(const void* acc, const double* terms, int nterms) {
  const xacc_t* s = (const xacc_t*)acc;
  xacc_t d;
  memset(&d, 0, sizeof d);
  for (int k = 0; k < nterms; k++) xacc_add_f64(&d, terms[k], 0);
  xacc_t negs = *s;
  xacc_carry(&negs);
  for (int i = 0; i < XACC_NDIG; i++) negs.dig[i] = -negs.dig[i];
  negs.nan = s->nan;
  negs.pinf = s->ninf; /* -S swaps the infinities */
  negs.ninf = s->pinf;
  xacc_merge(&d, &negs);
  return round_value(&d, 53, -1074);
}

int oracle_xacc_sign(const void* acc) {
  const xacc_t* s = (const xacc_t*)acc;
  if (s->nan || s->pinf || s->ninf) return 0;
  xacc_t m;
  int neg = xacc_magnitude(s, &m);
  for (int i = 0; i < XACC_NDIG; i++)
    if (m.dig[i]) return neg ? -1 : 1;
  return 0;
}
