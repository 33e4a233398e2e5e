/*
 * paper_loops.c: the paper's sequential summation loops in binary32 and
 * binary64 (test infrastructure, see twofold_oracle.h).
 */
#include <math.h>
#include <stdint.h>

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
