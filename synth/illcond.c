/*
 * illcond.c: second half of the ill-conditioned dot-product inputs.
 *
 * Input generator only: it makes data, it computes no result of the
 * summation methods. The running dot P of the elements generated so far is
 * kept in x87 extended precision (long double, 64-bit significand): the
 * products of two binary32 numbers are exact there, those of two binary64
 * numbers round at 2^-64 relative, which is ample for steering the
 * cancellation. Each new y_i is chosen so that x_i*y_i cancels P toward
 * m'_i * 2^(e_i):
 *     y_i = fl_T((m'_i * 2^e_i - P) / x_i)      (quotient in extended)
 * and e_i decays linearly from hi_exp to 0 over the second half.
 */
#include <math.h>
#include <stdint.h>

/* Exponent of element i of the second half [n0, n): hi_exp at i = n0,
 * 0 at i = n - 1, rounded to nearest (ties away from zero). */
static int decay_exp(int64_t i, int64_t n0, int64_t n, int hi_exp) {
  if (n - 1 <= n0) return 0;
  double f = (double)hi_exp * (double)(n - 1 - i) / (double)(n - 1 - n0);
  return (int)floor(f + 0.5);
}

/* mx, my: the uniform(-1,1) mantissas for elements n0..n-1 (binary64
 * holding values of the data type). x[0..n0) and y[0..n0) are already
 * filled. Returns the number of products whose magnitude fell below
 * tiny (a nonzero product that small could lose its FMA remainder to
 * underflow); callers require 0. *p_final receives the final running dot
 * rounded to binary64, an estimate used only to calibrate the recipe. */
int64_t synth_illcond_tail_f64(double* x, double* y, int64_t n0, int64_t n, const double* mx,
                               const double* my, int hi_exp, double tiny, double* p_final) {
  long double P = 0;
  for (int64_t i = 0; i < n0; i++) P += (long double)x[i] * (long double)y[i];
  int64_t small = 0;
  for (int64_t i = n0; i < n; i++) {
    int e = decay_exp(i, n0, n, hi_exp);
    double xi = ldexp(mx[i - n0], e);
    double target = ldexp(my[i - n0], e);
    double yi;
    if (xi == 0)
      yi = target;
    else
      yi = (double)(((long double)target - P) / (long double)xi);
    x[i] = xi;
    y[i] = yi;
    long double p = (long double)xi * (long double)yi;
    if (p != 0 && fabs((double)p) < tiny) small++;
    P += p;
  }
  *p_final = (double)P;
  return small;
}

int64_t synth_illcond_tail_f32(float* x, float* y, int64_t n0, int64_t n, const double* mx,
                               const double* my, int hi_exp, double tiny, double* p_final) {
  long double P = 0;
  for (int64_t i = 0; i < n0; i++) P += (long double)x[i] * (long double)y[i];
  int64_t small = 0;
  for (int64_t i = n0; i < n; i++) {
    int e = decay_exp(i, n0, n, hi_exp);
    float xi = (float)ldexp(mx[i - n0], e);
    float target = (float)ldexp(my[i - n0], e);
    float yi;
    if (xi == 0)
      yi = target;
    else
      yi = (float)(((long double)target - P) / (long double)xi);
    x[i] = xi;
    y[i] = yi;
    long double p = (long double)xi * (long double)yi;
    if (p != 0 && fabs((double)p) < tiny) small++;
    P += p;
  }
  *p_final = (double)P;
  return small;
}
