/*
 * dw.h: double-word (double-double) additions for the oracle (test
 * infrastructure). A double-word number is a pair (h, l) of binary64
 * numbers with h = fl(h + l), standing for h + l. The two additions are the
 * published algorithms of Joldes, Muller and Popescu, "Tight and rigorous
 * error bounds for basic building blocks of double-word arithmetic" (ACM
 * Transactions on Mathematical Software 44(2), 2017):
 *   DWPlusFP (their Algorithm 4): relative error at most 2u^2;
 *   AccurateDWPlusDW (their Algorithm 6): relative error at most
 *   3u^2 + 13u^3;
 * built from two-sum (the paper's Theorem 2, Knuth) and fast-two-sum
 * (Theorem 1, Dekker). Used for the wider accumulator on binary64 data, the
 * stand-in for the paper's quad accumulator. Compiled without contraction.
 */
#ifndef ORACLE_DW_H
#define ORACLE_DW_H

/* s + d = a + b exactly, s = fl(a + b) (Knuth). */
static inline void dw_two_sum(double a, double b, double* s, double* d) {
  double x = a + b;
  double bv = x - a;
  double av = x - bv;
  *s = x;
  *d = (a - av) + (b - bv);
}

/* s + d = a + b exactly when exponent(a) >= exponent(b) (Dekker). */
static inline void dw_fast_two_sum(double a, double b, double* s, double* d) {
  double x = a + b;
  *s = x;
  *d = b - (x - a);
}

/* DWPlusFP: (h, l) + y. */
static inline void dw_plus_fp(double h, double l, double y, double* zh, double* zl) {
  double sh, sl;
  dw_two_sum(h, y, &sh, &sl);
  double v = l + sl;
  dw_fast_two_sum(sh, v, zh, zl);
}

/* AccurateDWPlusDW: (xh, xl) + (yh, yl). */
static inline void dw_plus_dw(double xh, double xl, double yh, double yl, double* zh,
                              double* zl) {
  double sh, sl, th, tl, vh, vl;
  dw_two_sum(xh, yh, &sh, &sl);
  dw_two_sum(xl, yl, &th, &tl);
  double c = sl + th;
  dw_fast_two_sum(sh, c, &vh, &vl);
  double w = tl + vl;
  dw_fast_two_sum(vh, w, zh, zl);
}

#endif
