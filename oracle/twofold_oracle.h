/*
 * twofold_oracle.h: CPU oracle for twofold summation and dot products.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library. The GPU library never includes,
 * links or calls it, and it shares no code with the GPU library.
 *
 * Everything here is plain sequential C compiled with strict IEEE semantics
 * (gcc -O2 -ffp-contract=off, SSE2, no fast-math), round to nearest even.
 *
 * Three parts:
 *   1. An exact fixed-point accumulator (xacc) that defines the target
 *      S = sum x_n or S = sum x_n*y_n exactly, and A = sum |x_n| or
 *      sum |x_n*y_n| exactly; results are rounded once, to nearest even.
 *   2. The paper's sequential methods (Latkin, "Twofold fast summation",
 *      section "Algorithms": Example 1 sumtf, Example 2 Kahan sumk,
 *      Example 3 sumt and direct sum, the double-accumulator sumd, and dot
 *      products that sum the rounded products x_i*y_i as items), restated
 *      on fast-two-sum and two-sum (Theorems 1 and 2); plus the dot with an
 *      FMA exact product (this library's reading, see the model below).
 *   3. An order model: the same per-element steps applied in the order the
 *      GPU library documents for its reductions, used for bitwise checks.
 */
#ifndef TWOFOLD_ORACLE_H
#define TWOFOLD_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- 1. exact accumulator ------------------------------------------------
 * Opaque buffer of oracle_xacc_size() bytes, owned by the caller.
 * add_* functions add exactly; abs_values != 0 adds |term| instead of term.
 * nthreads <= 1 runs on the calling thread; otherwise the range is split into
 * nthreads slices, each summed into its own accumulator and merged by integer
 * addition (so the result does not depend on nthreads).
 * Non-finite terms set a flag; rounding then returns NaN or +-Inf.        */
size_t oracle_xacc_size(void);
void   oracle_xacc_clear(void* acc);
void   oracle_xacc_add_sum_f32(void* acc, const float* x, int64_t n, int abs_values, int nthreads);
void   oracle_xacc_add_sum_f64(void* acc, const double* x, int64_t n, int abs_values, int nthreads);
void   oracle_xacc_add_dot_f32(void* acc, const float* x, const float* y, int64_t n, int abs_values, int nthreads);
void   oracle_xacc_add_dot_f64(void* acc, const double* x, const double* y, int64_t n, int abs_values, int nthreads);
/* Round the exact value to a binary format with prec_bits significand bits
 * and minimum (subnormal) exponent emin_sub (the weight of the smallest
 * subnormal): (53, -1074) for binary64, (24, -149) for binary32. */
double oracle_xacc_round(const void* acc, int prec_bits, int emin_sub);
/* fl64( sum(terms[0..nterms)) - S ): one rounding of an exact difference. */
double oracle_xacc_round_diff(const void* acc, const double* terms, int nterms);
/* Sign of the exact value: -1, 0 or +1 (0 also when non-finite). */
int    oracle_xacc_sign(const void* acc);

/* ---- 2. sequential loops of the paper (binary32 and binary64) -----------
 * out2 receives {value, error}. Functions without out2 return the sum.    */
float  oracle_sum_f32(const float* x, int64_t n);
float  oracle_sumk_f32(const float* x, int64_t n);
void   oracle_sumk_pair_f32(const float* x, int64_t n, float* out2);
void   oracle_sumtf_f32(const float* x, int64_t n, float* out2);
void   oracle_sumt_f32(const float* x, int64_t n, float* out2);
double oracle_sumd_f32(const float* x, int64_t n);
float  oracle_dot_f32(const float* x, const float* y, int64_t n);
float  oracle_dotk_f32(const float* x, const float* y, int64_t n);
void   oracle_dotk_pair_f32(const float* x, const float* y, int64_t n, float* out2);
void   oracle_dottf_rounded_f32(const float* x, const float* y, int64_t n, float* out2);
void   oracle_dott_rounded_f32(const float* x, const float* y, int64_t n, float* out2);
void   oracle_dottf_f32(const float* x, const float* y, int64_t n, float* out2);
void   oracle_dott_f32(const float* x, const float* y, int64_t n, float* out2);
double oracle_dotd_f32(const float* x, const float* y, int64_t n);
/* The wider accumulator for binary64 data: double-word (h, l) in place of
 * the paper's quad (see dw.h); out2 = {h, l}. */
void   oracle_sumdd_f64(const double* x, int64_t n, double* out2);
void   oracle_dotdd_f64(const double* x, const double* y, int64_t n, double* out2);
void   oracle_dw_plus_fp(double h, double l, double y, double* out2);
void   oracle_dw_plus_dw(double xh, double xl, double yh, double yl, double* out2);

double oracle_sum_f64(const double* x, int64_t n);
double oracle_sumk_f64(const double* x, int64_t n);
void   oracle_sumk_pair_f64(const double* x, int64_t n, double* out2);
void   oracle_sumtf_f64(const double* x, int64_t n, double* out2);
void   oracle_sumt_f64(const double* x, int64_t n, double* out2);
double oracle_dot_f64(const double* x, const double* y, int64_t n);
double oracle_dotk_f64(const double* x, const double* y, int64_t n);
void   oracle_dotk_pair_f64(const double* x, const double* y, int64_t n, double* out2);
void   oracle_dottf_rounded_f64(const double* x, const double* y, int64_t n, double* out2);
void   oracle_dott_rounded_f64(const double* x, const double* y, int64_t n, double* out2);
void   oracle_dottf_f64(const double* x, const double* y, int64_t n, double* out2);
void   oracle_dott_f64(const double* x, const double* y, int64_t n, double* out2);

/* ---- 3. order model --------------------------------------------------------
 * mode: 0 plain, 1 fast, 2 rigorous, 3 wide (the paper's sumd/dotd:
 * binary64 accumulator for binary32 data, double-word accumulator for
 * binary64 data), 4 Kahan (Example 2; the error is the
 * negated correction), 5 fast and 6 rigorous with the rounded product as
 * the item (the paper's dot rule; dots only). dtype: 4 (binary32) or 8
 * (binary64).
 * y == NULL selects the sum, otherwise the dot.
 * x_misalign: (address of x modulo 16) / dtype, i.e. where x starts inside
 * its 16-byte line, in elements (0 .. 16/dtype - 1). The head of a range
 * starting at element o is the number of elements before the next 16-byte
 * boundary: (W - (x_misalign + o) mod W) mod W, capped at the range length,
 * with W = 16/dtype.
 * out2: {value, error} as binary64 (the binary32 results widen exactly).
 * viol (may be NULL): for the fast forms (1, 5), the sum of |item| over the
 * per-lane steps where Theorem 1's condition |s| >= |item| fails with
 * s != 0, in binary64; +0 for the other modes. Only those steps can lose
 * part of their round-off, each at most u(1 + 2u)|item|.
 * Returns 0, or -1 for invalid arguments or allocation failure.           */
int oracle_model_single(int dtype, int mode, const void* x, const void* y, int64_t n,
                        int x_misalign, int block_threads, int unroll, int grid_blocks,
                        double* out2, double* viol);
/* Segmented order model. offsets[0..nseg] (int64, non-decreasing), element
 * offsets into x (and y). tile_elems must be a multiple of 64*16/dtype.
 * Which wave processes which tile does not change any bit of the result
 * (a tile's pair depends only on its elements, and the tiles of a segment
 * are combined in tile order), so grid and block sizes are not inputs.
 * out: 2*nseg doubles, {value, error} per segment. viol (may be NULL):
 * nseg doubles, the single-vector model's viol per segment. */
int oracle_model_seg(int dtype, int mode, const void* x, const void* y,
                     const int64_t* offsets, int64_t nseg, int x_misalign,
                     int unroll, int64_t tile_elems, double* out, double* viol);

#ifdef __cplusplus
}
#endif
#endif
