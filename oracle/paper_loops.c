/*
 * paper_loops.c: the paper's sequential summation loops in binary32 and
 * binary64 (test infrastructure, see twofold_oracle.h).
 */
#include <math.h>
#include <stdint.h>

#include "dw.h"
#include "twofold_oracle.h"

#define T float
#define NAME(base) oracle_##base##_f32
#define FMA fmaf
#include "paper_loops.inc"
#undef T
#undef NAME
#undef FMA

#define T double
#define NAME(base) oracle_##base##_f64
#define FMA fma
#include "paper_loops.inc"
#undef T
#undef NAME
#undef FMA

/* Summation of binary32 data into a binary64 accumulator ("Algorithms",
 * the sumd function): each item is widened, which is exact. */
double oracle_sumd_f32(const float* x, int64_t n) {
  double s = 0;
  for (int64_t i = 0; i < n; i++) s = s + (double)x[i];
  return s;
}

/* The dot counterpart: both factors are widened before multiplying, so the
 * binary64 product of two binary32 numbers is exact (48 significant bits). */
double oracle_dotd_f32(const float* x, const float* y, int64_t n) {
  double s = 0;
  for (int64_t i = 0; i < n; i++) {
    double p = (double)x[i] * (double)y[i];
    s = s + p;
  }
  return s;
}

/* The wider accumulator for binary64 data. The paper's sumd/dotd on double
 * data accumulate in quad precision; here a double-word accumulator
 * (h, l) stands in for it (dw.h): each item enters with DWPlusFP, each dot
 * term as the exact product p + pi with AccurateDWPlusDW. out2 = {h, l}. */
void oracle_sumdd_f64(const double* x, int64_t n, double* out2) {
  double h = 0, l = 0;
  for (int64_t i = 0; i < n; i++) dw_plus_fp(h, l, x[i], &h, &l);
  out2[0] = h;
  out2[1] = l;
}

void oracle_dotdd_f64(const double* x, const double* y, int64_t n, double* out2) {
  double h = 0, l = 0;
  for (int64_t i = 0; i < n; i++) {
    double p = x[i] * y[i];
    double pi = fma(x[i], y[i], -p);
    dw_plus_dw(h, l, p, pi, &h, &l);
  }
  out2[0] = h;
  out2[1] = l;
}

/* The two double-word additions on their own, for the step pins. */
void oracle_dw_plus_fp(double h, double l, double y, double* out2) {
  dw_plus_fp(h, l, y, &out2[0], &out2[1]);
}

void oracle_dw_plus_dw(double xh, double xl, double yh, double yl, double* out2) {
  dw_plus_dw(xh, xl, yh, yl, &out2[0], &out2[1]);
}
