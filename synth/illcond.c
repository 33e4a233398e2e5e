/*
 * illcond.c: second half of the ill-conditioned dot-product inputs.
 *
 * Input generator only: it makes data, it computes no result of the
 * summation methods. The running dot P of the elements generated so far is
 * kept in binary128 (__float128): products of two binary64 (or binary32)
 * numbers are exact there, and the sum rounds at 2^-113 relative. Each new
 * y_i is chosen so that x_i*y_i cancels P toward m'_i * 2^(e_i):
 *     y_i = fl_T((m'_i * 2^e_i - P) / x_i)      (quotient in binary128)
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
  __float128 P = 0;
  for (int64_t i = 0; i < n0; i++) P += (__float128)x[i] * (__float128)y[i];
  int64_t small = 0;
  for (int64_t i = n0; i < n; i++) {
    int e = decay_exp(i, n0, n, hi_exp);
    double xi = ldexp(mx[i - n0], e);
    double target = ldexp(my[i - n0], e);
    double yi;
    if (xi == 0)
      yi = target;
    else
      yi = (double)(((__float128)target - P) / (__float128)xi);
    x[i] = xi;
    y[i] = yi;
    __float128 p = (__float128)xi * (__float128)yi;
    if (p != 0 && fabs((double)p) < tiny) small++;
    P += p;
  }
  *p_final = (double)P;
  return small;
}

int64_t synth_illcond_tail_f32(float* x, float* y, int64_t n0, int64_t n, const double* mx,
                               const double* my, int hi_exp, double tiny, double* p_final) {
  __float128 P = 0;
  for (int64_t i = 0; i < n0; i++) P += (__float128)x[i] * (__float128)y[i];
  int64_t small = 0;
  for (int64_t i = n0; i < n; i++) {
    int e = decay_exp(i, n0, n, hi_exp);
    float xi = (float)ldexp(mx[i - n0], e);
    float target = (float)ldexp(my[i - n0], e);
    float yi;
    if (xi == 0)
      yi = target;
    else
      yi = (float)(((__float128)target - P) / (__float128)xi);
    x[i] = xi;
    y[i] = yi;
    __float128 p = (__float128)xi * (__float128)yi;
    if (p != 0 && fabs((double)p) < tiny) small++;
    P += p;
  }
  *p_final = (double)P;
  return small;
}
