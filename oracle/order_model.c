/*
 * order_model.c: the GPU library's documented reduction order, replayed on
 * the CPU (test infrastructure, see twofold_oracle.h).
 *
 * The per-element steps are the paper's (Examples 1 and 3, and the dot rule
 * with an FMA remainder); what this file adds is only the ORDER in which the
 * GPU library applies them, as its public header describes it:
 *
 * Single vector, launch (BT threads per block, U vectors per lane per
 * round, GB blocks), L = GB*BT lanes, W = 16/sizeof(T) elements per vector:
 *   1. head: the h elements before x's first 16-byte boundary, element i on
 *      lane i, chain 0;
 *   2. body: V = floor((n-h)/W) vectors; in round q, lane g takes vectors
 *      q*U*L + u*L + g for u = 0..U-1, component j on chain j;
 *   3. tail: the r = n-h-V*W last elements, element i of them on lane i,
 *      chain 0;
 *   4. each lane merges chains 0..W-1 in order;
 *   5. each 64-lane wave combines with xor partners 1, 2, 4, 8, 16, 32;
 *   6. each block combines its waves' pairs in wave order;
 *   7. with one block its pair is the result; otherwise the GB block pairs,
 *      widened to binary64, go to 256 lanes (lane l takes l, l+256, ... in
 *      order, starting from +0), then steps 5 and 6 in binary64;
 *   8. finalize: binary64 results as they are; binary32 value fl32(V) and
 *      error fl32((V - value) + E), both operations in binary64 (error +0
 *      for the plain and wide modes, whose pairs carry no error).
 * The wide mode on binary64 data keeps double-word chains and combines
 * them with AccurateDWPlusDW in every step above (dw.h). The mixed mode
 * (binary32 data) keeps binary64 chains whose value is always a binary32
 * number: steps and combines before step 7 do the rigorous form's
 * arithmetic on the value in binary32 and add its exact remainders to the
 * binary64 error; step 7 is the binary64 combine; finalize gives value
 * fl32(V) and error (V - value) + E in binary64.
 * Segmented, tiles of TS elements (TS a multiple of 64*W): segment s has
 * ceil(len_s/TS) tiles; each tile is reduced by one 64-lane wave with
 * steps 1-5 on the tile's range; a one-tile segment's pair is finalized
 * directly; a longer segment's tile pairs, widened, go to 64 lanes (lane l
 * takes tiles l, l+64, ... in order, from +0), then step 5 in binary64,
 * then finalize; an empty segment gives (+0, +0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "dw.h"
#include "twofold_oracle.h"

#define MODE_PLAIN 0
#define MODE_FAST 1
#define MODE_RIGOROUS 2
#define MODE_WIDE 3
#define MODE_KAHAN 4
#define MODE_FAST_ROUNDED 5
#define MODE_RIGOROUS_ROUNDED 6
/* binary32 data only: the rigorous form with a binary64 error term */
#define MODE_MIXED 7
/* The wide mode on binary64 data: a double-word accumulator (dw.h). The
 * public mode number is MODE_WIDE for both data types; this one is the
 * model's own name for the binary64 case. */
#define MODE_DW 8
#define HAS_ERROR(m) ((m) != MODE_PLAIN && (m) != MODE_WIDE)

/* Two-sum (Theorem 2) in binary32, for the mixed mode's value chain. */
static void two_sum_b32(float a, float b, float* s, float* r) {
  float t = a + b;
  float bv = t - a;
  float av = t - bv;
  *s = t;
  *r = (a - av) + (b - bv);
}

static void combine64(int mode, double* s1, double* e1, double s2, double e2) {
  if (!HAS_ERROR(mode)) {
    *s1 = *s1 + s2;
    *e1 = 0;
    return;
  }
  if (mode == MODE_DW) {
    dw_plus_dw(*s1, *e1, s2, e2, s1, e1);
    return;
  }
  double a = *s1, b = s2;
  double x = a + b;
  double bp = x - a;
  double ap = x - bp;
  double bh = b - bp;
  double ah = a - ap;
  double y = ah + bh;
  *e1 = (*e1 + e2) + y;
  *s1 = x;
}

static void wave64(int mode, double* s, double* e) {
  double ns[64], ne[64];
  for (int d = 1; d < 64; d <<= 1) {
    for (int l = 0; l < 64; l++) {
      ns[l] = s[l];
      ne[l] = e[l];
      combine64(mode, &ns[l], &ne[l], s[l ^ d], e[l ^ d]);
    }
    for (int l = 0; l < 64; l++) {
      s[l] = ns[l];
      e[l] = ne[l];
    }
  }
}

/* Binary64 combine of count pairs by nlanes lanes (a multiple of 64):
 * strided sequential per lane, then per-wave xor combine, then waves in
 * order. */
static void grid_combine64(int mode, const double* ps, const double* pe, int64_t count,
                           int nlanes, double* V, double* E) {
  double s[1024], e[1024];
  for (int l = 0; l < nlanes; l++) {
    s[l] = 0.0;
    e[l] = 0.0;
    for (int64_t i = l; i < count; i += nlanes) combine64(mode, &s[l], &e[l], ps[i], pe[i]);
  }
  for (int w = 0; w < nlanes / 64; w++) wave64(mode, &s[w * 64], &e[w * 64]);
  double rs = s[0], re = e[0];
  for (int w = 1; w < nlanes / 64; w++) combine64(mode, &rs, &re, s[w * 64], e[w * 64]);
  *V = rs;
  *E = re;
}

static void finalize(int mode, int tsize, double V, double E, double* out2) {
  if (tsize == 8 || mode == MODE_WIDE) {
    out2[0] = V;
    out2[1] = E;
    return;
  }
  if (mode == MODE_MIXED) {
    /* value fl32(V); the error stays binary64: (V - value) + E */
    double v = (double)(float)V;
    out2[0] = v;
    out2[1] = (V - v) + E;
    return;
  }
  float v = (float)V;
  float e = 0.0f;
  if (HAS_ERROR(mode)) {
    double rest = V - (double)v; /* exact: V and v share their leading bits */
    e = (float)(rest + E);
  }
  out2[0] = (double)v;
  out2[1] = (double)e;
}

#define T float
#define A float
#define FMA_T fmaf
#define NAME(base) m32_##base
#include "order_model.inc"
#undef T
#undef A
#undef FMA_T
#undef NAME

#define T double
#define A double
#define FMA_T fma
#define NAME(base) m64_##base
#define WITH_DW 1
#include "order_model.inc"
#undef WITH_DW
#undef T
#undef A
#undef FMA_T
#undef NAME

/* binary32 data, binary64 accumulators (modes WIDE and MIXED). */
#define T float
#define A double
#define FMA_T fmaf
#define NAME(base) mw_##base
#include "order_model.inc"
#undef T
#undef A
#undef FMA_T
#undef NAME

static int valid_common(int dtype, int mode, int is_dot, int U) {
  if (dtype != 4 && dtype != 8) return 0;
  if (mode < MODE_PLAIN || mode > MODE_MIXED) return 0;
  if (mode == MODE_MIXED && dtype != 4) return 0;
  if ((mode == MODE_FAST_ROUNDED || mode == MODE_RIGOROUS_ROUNDED) && !is_dot) return 0;
  if (U < 1 || U > 64) return 0;
  return 1;
}

int oracle_model_single(int dtype, int mode, const void* x, const void* y, int64_t n,
                        int x_misalign, int block_threads, int unroll, int grid_blocks,
                        double* out2, double* viol) {
  if (!valid_common(dtype, mode, y != NULL, unroll) || n < 0 || (!x && n > 0)) return -1;
  if (block_threads < 64 || block_threads > 1024 || block_threads % 64) return -1;
  if (grid_blocks < 1 || (int64_t)grid_blocks * block_threads > ((int64_t)1 << 26)) return -1;
  if (x_misalign < 0 || x_misalign >= 16 / dtype) return -1;
  int is_dot = y != NULL;
  if (dtype == 8 && mode == MODE_WIDE) mode = MODE_DW;
  if (dtype == 8)
    return m64_single(mode, is_dot, (const double*)x, (const double*)y, n, x_misalign,
                      block_threads, unroll, grid_blocks, out2, viol);
  if (mode == MODE_WIDE || mode == MODE_MIXED)
    return mw_single(mode, is_dot, (const float*)x, (const float*)y, n, x_misalign,
                     block_threads, unroll, grid_blocks, out2, viol);
  return m32_single(mode, is_dot, (const float*)x, (const float*)y, n, x_misalign,
                    block_threads, unroll, grid_blocks, out2, viol);
}

int oracle_model_seg(int dtype, int mode, const void* x, const void* y,
                     const int64_t* offsets, int64_t nseg, int x_misalign,
                     int unroll, int64_t tile_elems, double* out, double* viol) {
  if (!valid_common(dtype, mode, y != NULL, unroll) || nseg < 0 || !offsets) return -1;
  if (tile_elems <= 0 || tile_elems % (64 * (16 / dtype))) return -1;
  if (x_misalign < 0 || x_misalign >= 16 / dtype) return -1;
  if (nseg > 0 && offsets[0] < 0) return -1;
  for (int64_t s = 0; s < nseg; s++)
    if (offsets[s + 1] < offsets[s]) return -1;
  int is_dot = y != NULL;
  if (dtype == 8 && mode == MODE_WIDE) mode = MODE_DW;
  if (dtype == 8)
    return m64_seg(mode, is_dot, (const double*)x, (const double*)y, offsets, nseg, x_misalign,
                   unroll, tile_elems, out, viol);
  if (mode == MODE_WIDE || mode == MODE_MIXED)
    return mw_seg(mode, is_dot, (const float*)x, (const float*)y, offsets, nseg, x_misalign,
                  unroll, tile_elems, out, viol);
  return m32_seg(mode, is_dot, (const float*)x, (const float*)y, offsets, nseg, x_misalign,
                 unroll, tile_elems, out, viol);
}
