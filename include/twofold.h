/*
 * twofold.h: C interface of the gfx950 twofold summation library.
 *
 * Twofold summation (E. Latkin, "Twofold fast summation", 2013) returns a sum
 * sum x_n or a dot product sum x_n*y_n as a pair (value, error): value is
 * what plain floating-point summation computes, and error collects the
 * round-offs that summation made, so that value + error approximates the
 * exact result better than value alone ("Overview"; section "Algorithms",
 * the text after Example 2).
 *
 * Modes (section "Algorithms"):
 *   TWOFOLD_PLAIN     direct summation (Example 3, second function); error 0.
 *   TWOFOLD_FAST      fast twofold step built on Dekker's fast-two-sum
 *                     (Theorem 1, Example 1). Exact per step only when
 *                     |running sum| >= |item|; otherwise the step loses part
 *                     of its round-off (at most about u*|item|).
 *   TWOFOLD_RIGOROUS  rigorous twofold step built on Knuth's two-sum
 *                     (Theorem 2, Example 3): every step's round-off is
 *                     captured exactly.
 *   TWOFOLD_KAHAN     compensated summation (Example 2): value is the
 *                     compensated sum, error the correction still pending
 *                     (-c); pairs are combined like twofold pairs.
 *   TWOFOLD_FAST_ROUNDED, TWOFOLD_RIGOROUS_ROUNDED  dots only: the paper's
 *                     own dot rule, the rounded product as the item and its
 *                     rounding not tracked (same value as the FMA forms).
 *   TWOFOLD_MIXED     binary32 data only: the rigorous form with its error
 *                     term in binary64. The value is the binary32 rigorous
 *                     value, bit for bit; each step's exact round-off (a
 *                     binary32 number) is added to a binary64 error, so the
 *                     error term no longer rounds at binary32 precision.
 *                     Results are binary64 pairs (twofold_sum_mixed_f32,
 *                     twofold_dot_mixed_f32, plans). This mode uses binary64
 *                     arithmetic inside binary32 reductions, as the paper's
 *                     sumd/dotd comparators do.
 * Dot products: the paper substitutes the rounded product a[i]*b[i] for the
 * data item (end of "Algorithms"). This library also captures the product's
 * rounding: p = fl(x*y), pi = fma(x, y, -p), x*y = p + pi exactly unless the
 * product underflows; p is the item and pi joins the error
 * (fast: e += pi - c; rigorous: e += (ds + dy) + pi).
 * The paper's sumd/dotd (a wider accumulator, section "Performance",
 * function list) are twofold_sumd_* / twofold_dotd_* (mode TWOFOLD_WIDE):
 * binary32 data summed in binary64 as the paper does, and binary64 data,
 * for which the paper used quad precision, summed in double-word
 * (double-double) arithmetic: the accumulator (h, l) takes each item with
 * DWPlusFP, or each exact product p + pi with AccurateDWPlusDW, and pairs
 * combine with AccurateDWPlusDW (Joldes, Muller, Popescu, ACM TOMS 2017,
 * Algorithms 4 and 6); the result's value is h and its error l.
 *
 * All arithmetic is IEEE round-to-nearest-even with no contraction other
 * than the one FMA above; binary32 subnormals are kept. A twofold value is
 * bitwise the plain result of the same launch configuration.
 *
 * ---- Reduction order (normative: it fixes every bit of every result) -----
 * T is float or double, W = 16/sizeof(T) (elements per 16-byte vector).
 * Every chain starts at (+0, +0). combine((s1,e1),(s2,e2)) is two-sum
 * (Theorem 2, all six operations) of s1, s2 giving (x, y), then
 * error (e1 + e2) + y, value x; in plain and binary32 wide modes it is
 * (s1 + s2, +0); in binary64 wide mode it is AccurateDWPlusDW. The Kahan
 * step keeps e = -c: yk = item + e, t = s + yk, e = yk - (t - s), s = t
 * (exactly Example 2's operations, negated).
 * Single vector, launch (block_threads BT, unroll U, grid_blocks GB),
 * L = GB*BT lanes, lane g = block*BT + thread:
 *   1. head: the h = min(n, elements before x's first 16-byte boundary)
 *      first elements, element i on lane i, chain 0;
 *   2. body: V = floor((n-h)/W) vectors; round q gives lane g the vectors
 *      k = q*U*L + u*L + g, u = 0..U-1 in order (k < V), component j of
 *      vector k (element h + k*W + j) on chain j;
 *   3. tail: the r = n - h - V*W last elements, element i of them on lane
 *      i, chain 0;
 *   4. each lane combines its chains in order 0, 1, ..., W-1;
 *   5. each 64-lane wave: for d = 1, 2, 4, 8, 16, 32, lane l replaces its
 *      pair P_l by combine(P_l, P_{l xor d}) (pairs as before the step);
 *   6. each block combines its waves' lane-0 pairs in wave order;
 *   7. if GB = 1 the block pair is the result R; otherwise R is computed in
 *      binary64 from the GB block pairs (widened exactly): 256 lanes, lane
 *      l starting at (+0,+0) and combining pairs l, l+256, ... in order,
 *      then steps 5 and 6 over those 256 lanes;
 *   8. finalize R = (V, E): binary64 results are (V, E); binary32 results
 *      are value fl32(V) and error fl32((V - value) + E), in binary64
 *      (V - value is exact); plain and wide results have error +0.
 * Segmented, launch (block_threads, unroll U, grid_blocks, tile_elems TS):
 *   segment s covers elements [off[s], off[s+1]) and has ceil(len/TS)
 *   tiles; tile j covers [off[s] + j*TS, min(off[s+1], off[s] + (j+1)*TS));
 *   each tile is reduced by one 64-lane wave with steps 1-5 applied to the
 *   tile's range (L = 64); a one-tile segment's pair is finalized (step 8);
 *   the tile pairs of a longer segment are combined in binary64 by 64
 *   lanes, lane l starting at (+0,+0) and combining tiles l, l+64, ... in
 *   tile order, then step 5, then step 8; an empty segment gives (+0,+0).
 *   Which wave handles which tile does not change the result.
 * Multi-vector calls: vector v is reduced by steps 1-8 with the call's
 * launch, exactly as a single-vector call with that launch reduces it.
 * Mixed (binary32 data): chains and combines as the rigorous mode, with the
 * value in binary32 and the error in binary64: the step is t = s + item,
 * yt = t - s, dy = item - yt, ds = s - (t - yt) in binary32, then
 * e = e + (double)(ds + dy), for dots e = e + ((double)(ds + dy) +
 * (double)pi) with pi = fma(x, y, -p) in binary32; combine is the binary32
 * two-sum of the values (x, y) and e = (e1 + e2) + (double)y. Step 7 uses
 * the binary64 combine of the rigorous mode; step 8 gives value
 * fl32(V) and error (V - value) + E, both binary64.
 * Wide (sumd/dotd): binary32 data: as above with binary64 chains over
 * widened binary32 data and the plain combine; results are binary64 pairs
 * with error +0. binary64 data: as above with double-word chains: the step
 * (h, l) = DWPlusFP((h, l), x), for dots AccurateDWPlusDW((h, l), (p, pi))
 * with p = fl(x*y), pi = fma(x, y, -p); combine is AccurateDWPlusDW, written
 * out as (sh, sl) = two-sum(h1, h2), (th, tl) = two-sum(l1, l2),
 * c = sl + th, (vh, vl) = fast-two-sum(sh, c), w = tl + vl,
 * (h, l) = fast-two-sum(vh, w); DWPlusFP as (sh, sl) = two-sum(h, x),
 * v = l + sl, (h, l) = fast-two-sum(sh, v); fast-two-sum(a, b) is s = a + b,
 * (s, b - (s - a)).
 *
 * ---- Conventions --------------------------------------------------------
 * Pointers: x, y, out, offsets and ws are device pointers (hipMalloc or
 * torch device memory) on the current HIP device; the caller owns them.
 * Data pointers must be aligned to their element size (they may be NULL
 * when there are no elements); x and y may have different alignments within
 * a 16-byte line. stream is a hipStream_t
 * (NULL: the legacy default stream). Calls are asynchronous: results are in
 * out once the stream reaches them. The execute paths never allocate, free
 * or synchronise, and may be captured into a HIP graph.
 * Workspace: ws is device scratch of at least the bytes the matching
 * twofold_workspace_bytes_* call returns, 256-byte aligned; it needs no
 * preparation and holds nothing useful afterwards. Calls that may run at
 * the same time need separate workspaces. A single-vector call that runs
 * one block does not touch ws (it may then be NULL).
 * Kernels: a single-vector, multi-vector or batch call is one kernel (one
 * block) or two (blocks, then the binary64 combine); a segmented call is
 * three small tiling kernels (device offsets only: per-row tile counts, the
 * rows' prefix, then the tile and wave tables), the tile kernel and the
 * per-segment combine kernel. Later kernels see earlier ones' results through the
 * stream order alone: no kernel waits on, or fences for, another block.
 * Status: 0 on success, a negative TWOFOLD_E* code otherwise; arguments are
 * checked on the host before any HIP call, and nothing is launched on
 * error. Non-finite inputs give IEEE values and an unspecified error.
 * Element counts (n, n_total, nseg, offsets[nseg]) are at most 2^56.
 */
#ifndef TWOFOLD_H
#define TWOFOLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The pair type of the paper's Example 1 (struct twofold<number>). */
typedef struct { float value, error; } twofold_f32_t;
typedef struct { double value, error; } twofold_f64_t;

enum {
  TWOFOLD_PLAIN = 0,
  TWOFOLD_FAST = 1,
  TWOFOLD_RIGOROUS = 2,
  TWOFOLD_WIDE = 3, /* the wider accumulator (sumd/dotd, plans): binary64 for
                       binary32 data, double-word for binary64 data */
  TWOFOLD_KAHAN = 4,
  TWOFOLD_FAST_ROUNDED = 5,
  TWOFOLD_RIGOROUS_ROUNDED = 6,
  TWOFOLD_MIXED = 7
};

enum {
  TWOFOLD_OK = 0,
  TWOFOLD_EINVAL = -1,     /* bad pointer, size, mode or launch value    */
  TWOFOLD_EWORKSPACE = -2, /* workspace missing or too small             */
  TWOFOLD_EHIP = -3,       /* a HIP call failed (launch or runtime)      */
  TWOFOLD_EALIGN = -4,     /* a data pointer is not element-aligned      */
  TWOFOLD_EOFFSETS = -5,   /* segment offsets not non-decreasing from 0.. */
  TWOFOLD_ENOTUNED = -6,   /* twofold_tuned_launch: no measured row      */
  TWOFOLD_ECAPTURE = -7    /* a stream capture is under way: plan
                              creation (synchronous) is not allowed      */
};

/* Launch configuration. Zero fields take the tuned default.
 *   block_threads: threads per block, 64..1024 in steps of 64.
 *   unroll:        vectors per lane per round: 1, 2, 4 or 8.
 *   grid_blocks:   single vector: exactly this many blocks, 1..1048576;
 *                  segmented: persistent blocks, 1..1048576.
 *   tile_elems:    segmented only: tile length, a positive multiple of
 *                  64*16/sizeof(T), at most 2^30.                        */
typedef struct {
  int32_t block_threads;
  int32_t unroll;
  int32_t grid_blocks;
  int32_t reserved; /* must be 0 */
  int64_t tile_elems;
} twofold_launch_t;

/* Fill *out with the configuration a call with launch == NULL uses:
 * kind 0 single vector (n elements), 1 segmented (n total elements,
 * nseg segments: the table's segmented rows are chosen by n and by the
 * mean segment length n / nseg, short segments having rows of their own).
 * dtype 4 or 8; mode TWOFOLD_*. */
int twofold_default_launch(int kind, int dtype, int is_dot, int mode, int64_t n, int64_t nseg,
                           twofold_launch_t* out);

/* The same default, and whether it was measured: the launch table holds
 * rows measured by the autotuner per (kind, dtype, operation, mode, size
 * bucket). Returns TWOFOLD_OK when a row of this very (kind, dtype, is_dot,
 * mode) covers n, TWOFOLD_ENOTUNED when the default is borrowed (from the
 * rigorous mode's rows of the same data type and operation, or the
 * built-in shape); *out is filled either way. Other errors as
 * twofold_default_launch. */
int twofold_tuned_launch(int kind, int dtype, int is_dot, int mode, int64_t n, int64_t nseg,
                         twofold_launch_t* out);

/* Workspace size for a single-vector call, and for a segmented call with
 * nseg segments over n_total elements. launch NULL: the default. */
size_t twofold_workspace_bytes_single(int dtype, int is_dot, int mode, int64_t n,
                                      const twofold_launch_t* launch);
size_t twofold_workspace_bytes_seg(int dtype, int is_dot, int mode, int64_t n_total, int64_t nseg,
                                   const twofold_launch_t* launch);

/* ---- single vector: one (value, error) pair into *out (device) ---------
 * Section "Algorithms": sumtf (Example 1), sumt and sum (Example 3), dot by
 * substitution of x[i]*y[i]; mode selects the form. n >= 0; n = 0 gives
 * (+0, +0). */
int twofold_sum_f32(const float* x, int64_t n, int mode, const twofold_launch_t* launch,
                    twofold_f32_t* out, void* ws, size_t ws_bytes, void* stream);
int twofold_sum_f64(const double* x, int64_t n, int mode, const twofold_launch_t* launch,
                    twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream);
int twofold_dot_f32(const float* x, const float* y, int64_t n, int mode,
                    const twofold_launch_t* launch, twofold_f32_t* out, void* ws, size_t ws_bytes,
                    void* stream);
int twofold_dot_f64(const double* x, const double* y, int64_t n, int mode,
                    const twofold_launch_t* launch, twofold_f64_t* out, void* ws, size_t ws_bytes,
                    void* stream);
/* Paper's sumd / dotd: binary32 data summed into binary64 (products of two
 * binary32 numbers are exact in binary64). out->error is +0. */
int twofold_sumd_f32(const float* x, int64_t n, const twofold_launch_t* launch,
                     twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream);
int twofold_dotd_f32(const float* x, const float* y, int64_t n, const twofold_launch_t* launch,
                     twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream);
/* The same for binary64 data, in double-word arithmetic (the paper's quad
 * accumulator, see above): out = (h, l), h + l the double-word sum. */
int twofold_sumd_f64(const double* x, int64_t n, const twofold_launch_t* launch,
                     twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream);
int twofold_dotd_f64(const double* x, const double* y, int64_t n, const twofold_launch_t* launch,
                     twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream);
/* Mode TWOFOLD_MIXED on binary32 data (see the modes above): out->value is
 * the binary32 rigorous value, out->error the binary64 error term. */
int twofold_sum_mixed_f32(const float* x, int64_t n, const twofold_launch_t* launch,
                          twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream);
int twofold_dot_mixed_f32(const float* x, const float* y, int64_t n,
                          const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                          size_t ws_bytes, void* stream);

/* ---- several vectors in one launch: count pairs into out[0..count) -------
 * x[v], y[v] (device data pointers) and n[v] (lengths) are HOST arrays of
 * count entries, 0 <= count <= 64; the vectors need not be contiguous, of
 * equal length or equally aligned. out[v] is bitwise the pair the
 * single-vector call (twofold_sum_* / twofold_dot_*) returns for vector v
 * with the same launch; launch NULL takes the default launch of the longest
 * vector. All vectors go through one kernel: short ones (at most 64 MiB
 * read each) side by side with a set of grid_blocks blocks each, longer
 * ones in turn through one set. One combine kernel finishes them all, so
 * the per-call costs (kernel start and end, the combine kernel) are paid
 * once per batch.
 * Modes as the single-vector calls: twofold_multisum_* / twofold_multidot_*
 * take the modes whose results have the data's type (TWOFOLD_WIDE and
 * TWOFOLD_MIXED give EINVAL there); the wider accumulator and the mixed form,
 * whose results are binary64 pairs, have their own calls below, each row
 * bitwise the matching sumd/dotd or mixed single-vector call. Workspace:
 * twofold_workspace_bytes_multi (count times the single-vector workspace of
 * the launch; mode TWOFOLD_WIDE or TWOFOLD_MIXED for the calls below); count
 * = 0 does nothing. */
size_t twofold_workspace_bytes_multi(int dtype, int is_dot, int mode, const int64_t* n,
                                     int64_t count, const twofold_launch_t* launch);
int twofold_multisum_f32(const float* const* x, const int64_t* n, int64_t count, int mode,
                         const twofold_launch_t* launch, twofold_f32_t* out, void* ws,
                         size_t ws_bytes, void* stream);
int twofold_multisum_f64(const double* const* x, const int64_t* n, int64_t count, int mode,
                         const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                         size_t ws_bytes, void* stream);
int twofold_multidot_f32(const float* const* x, const float* const* y, const int64_t* n,
                         int64_t count, int mode, const twofold_launch_t* launch,
                         twofold_f32_t* out, void* ws, size_t ws_bytes, void* stream);
int twofold_multidot_f64(const double* const* x, const double* const* y, const int64_t* n,
                         int64_t count, int mode, const twofold_launch_t* launch,
                         twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream);
int twofold_multisumd_f32(const float* const* x, const int64_t* n, int64_t count,
                          const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                          size_t ws_bytes, void* stream);
int twofold_multisumd_f64(const double* const* x, const int64_t* n, int64_t count,
                          const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                          size_t ws_bytes, void* stream);
int twofold_multidotd_f32(const float* const* x, const float* const* y, const int64_t* n,
                          int64_t count, const twofold_launch_t* launch, twofold_f64_t* out,
                          void* ws, size_t ws_bytes, void* stream);
int twofold_multidotd_f64(const double* const* x, const double* const* y, const int64_t* n,
                          int64_t count, const twofold_launch_t* launch, twofold_f64_t* out,
                          void* ws, size_t ws_bytes, void* stream);
int twofold_multisum_mixed_f32(const float* const* x, const int64_t* n, int64_t count,
                               const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                               size_t ws_bytes, void* stream);
int twofold_multidot_mixed_f32(const float* const* x, const float* const* y, const int64_t* n,
                               int64_t count, const twofold_launch_t* launch, twofold_f64_t* out,
                               void* ws, size_t ws_bytes, void* stream);

/* ---- a mixed batch: up to 64 sums and dots of either data type and any
 * form in one launch ---------------------------------------------------------
 * Each item names its data (device pointers), its length, its data type (4
 * or 8), whether it is a dot, its mode (any mode its single-vector calls
 * take) and its output pair: a device twofold_f32_t for binary32 data, a
 * twofold_f64_t for binary64 data and for TWOFOLD_WIDE and TWOFOLD_MIXED.
 * items is a HOST array. Every item's pair is bitwise the one its
 * single-vector call (twofold_sum_* / twofold_dot_*, twofold_sumd_* /
 * twofold_dotd_*, twofold_{sum,dot}_mixed_f32) returns with the batch's
 * launch; a batch with a TWOFOLD_WIDE or TWOFOLD_MIXED item runs a kernel
 * that holds those forms too. launch
 * NULL takes the default launch of the item that reads the most bytes, with
 * at most four vectors per lane a round (unroll <= 4) when that launch's
 * blocks have more than 512 threads. As in
 * the multi-vector calls, items of at most 64 MiB each run side by side,
 * longer ones in turn through one block set, and one combine kernel
 * finishes them all, so a batch pays the per-launch costs once.
 * Workspace: twofold_workspace_bytes_batch (count times the single-vector
 * workspace of the launch); count = 0 does nothing. */
typedef struct {
  const void* x;   /* device data, n elements of dtype bytes */
  const void* y;   /* device data for a dot; ignored for a sum */
  void* out;       /* device output pair: the data's type, binary64 for WIDE, MIXED */
  int64_t n;
  int32_t dtype;   /* 4: binary32, 8: binary64 */
  int32_t is_dot;  /* 0: sum of x, 1: dot of x and y */
  int32_t mode;    /* any mode of the single-vector calls (MIXED: binary32 data) */
  int32_t reserved;
} twofold_batch_item_t;
size_t twofold_workspace_bytes_batch(const twofold_batch_item_t* items, int64_t count,
                                     const twofold_launch_t* launch);
int twofold_batch(const twofold_batch_item_t* items, int64_t count,
                  const twofold_launch_t* launch, void* ws, size_t ws_bytes, void* stream);

/* twofold_batch without a workspace, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. Items, launch, stream and results are
 * those of twofold_batch (each pair bitwise twofold_batch's with the same
 * launch); nothing is allocated or freed and no allocating library routine
 * is called. The block pairs go to a static device array of
 * TWOFOLD_STATIC_SCRATCH_BYTES (4 MiB) that each device holds until the
 * process ends; the first call on a device looks its address up
 * (hipGetSymbolAddress) with that device current. A batch whose block pairs
 * need more (16 * count * grid_blocks bytes when grid_blocks > 1; e.g. 64
 * items of 4096 blocks) returns TWOFOLD_EWORKSPACE before any HIP call.
 * All calls on one device share the array and nothing in it outlives a
 * call: calls that can overlap on one device (on different streams, or
 * graphs replayed concurrently) race and must be ordered by the caller. */
#define TWOFOLD_STATIC_SCRATCH_BYTES (4u << 20)
int twofold_batch_static(const twofold_batch_item_t* items, int64_t count,
                         const twofold_launch_t* launch, void* stream);

/* ---- segmented (CSR) batches: nseg pairs into out[0..nseg) ---------------
 * offsets: device int64[nseg + 1], non-decreasing, offsets[0] >= 0 and
 * offsets[nseg] <= n_total (the length of x and y). Checked on the device:
 * on violation every out[s] is NaN.
 * twofold_segsum_f32 / twofold_segdot_f32 take the modes with binary32
 * results (TWOFOLD_WIDE and TWOFOLD_MIXED give EINVAL there); the _f64 calls
 * also take TWOFOLD_WIDE (double-word pairs). The binary64-result forms have
 * their own calls below: the wider accumulator (segsumd / segdotd, both
 * data types; for binary64 data the same as mode TWOFOLD_WIDE) and the
 * mixed form (binary32 data), out = binary64 pairs. */
int twofold_segsum_f32(const float* x, int64_t n_total, const int64_t* offsets, int64_t nseg,
                       int mode, const twofold_launch_t* launch, twofold_f32_t* out, void* ws,
                       size_t ws_bytes, void* stream);
int twofold_segsum_f64(const double* x, int64_t n_total, const int64_t* offsets, int64_t nseg,
                       int mode, const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                       size_t ws_bytes, void* stream);
int twofold_segdot_f32(const float* x, const float* y, int64_t n_total, const int64_t* offsets,
                       int64_t nseg, int mode, const twofold_launch_t* launch, twofold_f32_t* out,
                       void* ws, size_t ws_bytes, void* stream);
int twofold_segdot_f64(const double* x, const double* y, int64_t n_total, const int64_t* offsets,
                       int64_t nseg, int mode, const twofold_launch_t* launch, twofold_f64_t* out,
                       void* ws, size_t ws_bytes, void* stream);
int twofold_segsumd_f32(const float* x, int64_t n_total, const int64_t* offsets, int64_t nseg,
                        const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                        size_t ws_bytes, void* stream);
int twofold_segsumd_f64(const double* x, int64_t n_total, const int64_t* offsets, int64_t nseg,
                        const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                        size_t ws_bytes, void* stream);
int twofold_segdotd_f32(const float* x, const float* y, int64_t n_total, const int64_t* offsets,
                        int64_t nseg, const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                        size_t ws_bytes, void* stream);
int twofold_segdotd_f64(const double* x, const double* y, int64_t n_total, const int64_t* offsets,
                        int64_t nseg, const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                        size_t ws_bytes, void* stream);
int twofold_segsum_mixed_f32(const float* x, int64_t n_total, const int64_t* offsets,
                             int64_t nseg, const twofold_launch_t* launch, twofold_f64_t* out,
                             void* ws, size_t ws_bytes, void* stream);
int twofold_segdot_mixed_f32(const float* x, const float* y, int64_t n_total,
                             const int64_t* offsets, int64_t nseg, const twofold_launch_t* launch,
                             twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream);

/* ---- segmented plans: host offsets fixed once, one kernel per execute ---
 * create: validates offsets_host (host int64[nseg+1], offsets[0] = 0,
 * non-decreasing), builds the tile table and copies offsets and table to
 * device memory owned by the plan, with the plan's per-segment completion
 * (synchronous; not capturable). It returns TWOFOLD_ECAPTURE, and makes no
 * allocation or copy, when it finds a stream capture under way: on the
 * legacy default stream's view (a capture on any blocking stream), or
 * reported by the allocator (a global-mode capture on any stream). Create
 * plans before capturing; their executes are capturable. The workspace of
 * an execute holds the pairs of the tiles of multi-tile segments.
 * dtype 4 or 8; mode TWOFOLD_* (ROUNDED forms only for dots).
 * execute: the tile kernel (persistent waves) and the combine kernel on
 * stream, no host work in between; out is twofold_f64_t[nseg] for binary64
 * data and for modes WIDE and MIXED, twofold_f32_t[nseg] otherwise; y must
 * be NULL for sums and given for dots (is_dot at creation). Capturable.
 * A plan must not execute on two streams at once. */
typedef struct twofold_seg_plan twofold_seg_plan_t;
int twofold_seg_plan_create(const int64_t* offsets_host, int64_t nseg, int dtype, int is_dot,
                            int mode, const twofold_launch_t* launch, twofold_seg_plan_t** plan);
size_t twofold_seg_plan_workspace_bytes(const twofold_seg_plan_t* plan);
int twofold_seg_plan_get_launch(const twofold_seg_plan_t* plan, twofold_launch_t* out);
int twofold_seg_plan_execute(const twofold_seg_plan_t* plan, const void* x, const void* y,
                             void* out, void* ws, size_t ws_bytes, void* stream);
int twofold_seg_plan_destroy(twofold_seg_plan_t* plan);

/* ---- precision monitor ----------------------------------------------------
 * The paper proposes to stop a computation whose error term gets too large,
 * as a sign that the precision in use is not enough ("Algorithms", remarks
 * after the rigorous form), and expects twofold summation to work for N
 * below 1/u ("Overview"). twofold_monitor applies both to count results
 * already on the device:
 *   pairs:    device twofold_f32_t[count] (dtype 4) or twofold_f64_t[count]
 *             (dtype 8), e.g. the out array of a segmented call;
 *   offsets:  device int64[count + 1]; result i has length
 *             offsets[i+1] - offsets[i]. NULL: every result has length n;
 *   tau:      finite, >= 0;
 *   flags:    device uint32[count], written: TWOFOLD_FLAG_ERROR when
 *             |error| > tau*|value|, TWOFOLD_FLAG_LENGTH when the length is
 *             at least 1/u (2^24 for dtype 4, 2^53 for dtype 8),
 *             TWOFOLD_FLAG_NONFINITE when value or error is Inf or NaN (then
 *             TWOFOLD_FLAG_ERROR is not set). Comparisons are made in
 *             binary64 on the exactly widened pair, tau*|value| rounded once;
 *   nflagged: device int64, written: the number of nonzero flags.
 * Asynchronous on stream, no workspace, capturable (two kernels: one
 * clears *nflagged, one writes the flags and adds up the count). */
#define TWOFOLD_FLAG_ERROR 1u
#define TWOFOLD_FLAG_LENGTH 2u
#define TWOFOLD_FLAG_NONFINITE 4u
int twofold_monitor(int dtype, const void* pairs, int64_t count, const int64_t* offsets, int64_t n,
                    double tau, uint32_t* flags, int64_t* nflagged, void* stream);

/* ---- instruments ----------------------------------------------------------
 * Memory-only probe (the paper's read1/read2, section "Memory reading"):
 * streams x (and y, if not NULL), nbytes each, through the single-vector
 * sum's (dot's) own lane loop for launch (block_threads, unroll 1, 2, 4 or
 * 8, grid_blocks; every field required): the same 16-byte loads in the same
 * lane order, rounds and loads ahead, with the summation step replaced by a
 * bit-OR of the loaded 32-bit words. sink[b] (device uint64[grid_blocks])
 * receives the OR of every word block b loaded. x, y 16-byte aligned,
 * nbytes a multiple of 16. Its rate bounds what the reduction kernels can
 * stream with the same launch.                                          */
int twofold_probe_read(const void* x, const void* y, int64_t nbytes, const twofold_launch_t* launch,
                       uint64_t* sink, void* stream);
/* Compute-only probe (the paper's p-functions, section "Purely
 * computing"): every lane feeds 4*16/dtype register-resident items through
 * its chains iters times with the step of (dtype, is_dot, mode), 4 rounds
 * of W items per iteration. seed: device array of 64 elements of dtype;
 * sink: device double[2 * grid_blocks * block_threads].                 */
int twofold_probe_compute(int dtype, int is_dot, int mode, const void* seed, int64_t iters,
                          const twofold_launch_t* launch, double* sink, void* stream);

/* Static string for a status code. */
const char* twofold_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
