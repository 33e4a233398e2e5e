"""Error bounds for the GPU library's reduction trees (test infrastructure,
like the rest of this package).

The tolerance the tests apply everywhere is |v + e - S| <= 4 N u^2 sum|x y|.
That is a stated tolerance, not a theorem. For long sequential chains the
worst case grows like N^2 u^2 (a chain of length L carries L round-offs, each
up to u times a partial sum). This module gives the bound that holds for
the actual tree of a launch, derived below from Theorems 1 and 2. A result
above 4 N u^2 but below this bound is then a property of the tree, and a
result above this bound is a defect.

Derivation (rigorous form; u = unit round-off of the data type, which also
bounds the binary64 parts for binary32 data):

* Value path. Chains add items y (y = fl(x*y) for dots) into s; combines
  add pair values. Every rounding of the value path leaves an exact term:
  delta_i = round-off of s + y (Theorem 2; |delta_i| <= u |t_i|, t_i the
  computed partial sum), pi_i = fma remainder of a product (|pi_i| <= u |p_i|)
  and r_j = TWO-SUM remainder of combine j (|r_j| <= u |x_j|). With V the
  final value, S = V + sum(delta) + sum(pi) + sum(r) exactly.
* Sizes. A chain of at most Lc items has sum_i |t_i| <= Lc (1 + g(Lc)) sum|y|;
  an item lies under at most D combines, so sum_j |x_j| <= D (1 + g(Lc + D))
  sum|y|; and sum|y| <= (1 + u) A with A = sum|x y|. Hence the terms add up
  to at most T = u (Lc + D + 1) (1 + g(Lc + D)) (1 + u) A.
* Error path. The error e is the rounded sum of these terms: a term meets
  at most h = Lc + 2D + 3 roundings on its way to the output (one for
  (delta + pi), at most Lc chain additions, two per combine, two in the
  binary32 finalize). A summation tree of depth h errs by at most g(h) times
  the sum of the absolute terms, so |V + e - S| <= g(h) T.
* binary32 output: v = fl32(V) moves V - v (|V - v| <= u |V|) into the error
  before its last two roundings: add g(2) u (1 + g(Lc + D)) (1 + u) A.

g(k) = k u / (1 - k u). Fast form: a step that breaks Theorem 1's condition
loses rho with |rho| <= u (1 + 2u) |y|; with Sv the sum of |y| over those
steps (counted by the order model), the terms grow by at most
u (1 + 2u) Sv and the result moves by at most as much again.
"""
import math

import numpy as np

PASS2_LANES = 256  # lanes of the binary64 grid combine
WAVE_LEVELS = 6  # 64-lane butterfly


def unit_roundoff(dtype):
    return 2.0 ** -(np.finfo(dtype).nmant + 1)


def g(k, u):
    ku = k * u
    if ku >= 1:
        return math.inf
    return ku / (1 - ku)


def single_depths(dtype, n, block_threads, unroll, grid_blocks):
    """(Lc, D) of a single-vector launch: the most items any chain takes and
    the most combines any item passes through."""
    del unroll  # the rounds a lane runs do not change how many items it takes
    W = 16 // np.dtype(dtype).itemsize
    lanes = block_threads * grid_blocks
    vectors = n // W + 1  # an upper bound on the body vectors
    Lc = -(-vectors // lanes) + 2  # body, plus a head and a tail element
    D = (W - 1) + WAVE_LEVELS + (block_threads // 64 - 1)
    if grid_blocks > 1:
        D += -(-grid_blocks // PASS2_LANES) + WAVE_LEVELS + (PASS2_LANES // 64 - 1)
    return Lc, D


def segment_depths(dtype, seg_len, tile_elems):
    """(Lc, D) of one segment of a segmented launch (64-lane tiles)."""
    W = 16 // np.dtype(dtype).itemsize
    ntiles = -(-seg_len // tile_elems)
    Lc = -(-(tile_elems // W + 1) // 64) + 2
    D = (W - 1) + WAVE_LEVELS
    if ntiles > 1:
        D += -(-ntiles // 64) + WAVE_LEVELS
    return Lc, D


def tree_bound(dtype, Lc, D, A, fast_violations=0.0):
    """Bound on |v + e - S| for a tree of depths (Lc, D) over terms of
    absolute sum A (sum|x y| or sum|x|); fast_violations is the order model's
    violation sum for the fast forms (0 for the rigorous form)."""
    u = unit_roundoff(dtype)
    grow = (1 + g(Lc + D, u)) * (1 + u)
    loss = u * (1 + 2 * u) * fast_violations
    T = u * (Lc + D + 1) * grow * A + loss
    h = Lc + 2 * D + 3
    b = g(h, u) * T + loss
    if np.dtype(dtype) == np.float32:
        b += g(2, u) * u * grow * A
    return b


def single_bound(dtype, n, block_threads, unroll, grid_blocks, A, fast_violations=0.0):
    Lc, D = single_depths(dtype, n, block_threads, unroll, grid_blocks)
    return tree_bound(dtype, Lc, D, A, fast_violations)


def segment_bound(dtype, seg_len, tile_elems, A, fast_violations=0.0):
    Lc, D = segment_depths(dtype, seg_len, tile_elems)
    return tree_bound(dtype, Lc, D, A, fast_violations)


def dw_bound(Lc, D, A):
    """Bound on |h + l - S| for the wide mode on binary64 data (double-word
    chains and combines). Every double-word addition returns its operands'
    exact sum up to a relative 3u^2 + 13u^3 (AccurateDWPlusDW; DWPlusFP is
    within 2u^2), and an item lies under at most Lc + D additions (chain
    steps after it, then combines), so the errors add up to at most
    (Lc + D) (3u^2 + 13u^3) A, to first order; the denominator covers the
    errors' own growth."""
    u = unit_roundoff(np.float64)
    r = (Lc + D) * (3 * u * u + 13 * u ** 3)
    if r >= 1:
        return math.inf
    return r * A / (1 - r)


def mixed_bound(Lc, D, A):
    """Bound on |v + e - S| for the mixed mode (binary32 data, binary32
    value, binary64 error) over a tree of depths (Lc, D).

    The value path is the binary32 rigorous one, so its exact terms add up
    to at most T = u32 (Lc + D + 1) (1 + g32(Lc + D)) (1 + u32) A, as in
    tree_bound. They are summed in binary64: a term meets at most
    h = Lc + 2D + 3 binary64 roundings (one for the remainder plus the
    product remainder, Lc chain additions, two per combine, one in the
    finalize), so |V + E - S| <= g64(h) T. The finalize e = (V - v) + E
    rounds once more: at most u64 (|V - v| + |E|) <= u64 (u32 grow A +
    (1 + g64(h)) T)."""
    u32 = unit_roundoff(np.float32)
    u64 = unit_roundoff(np.float64)
    grow = (1 + g(Lc + D, u32)) * (1 + u32)
    T = u32 * (Lc + D + 1) * grow * A
    h = Lc + 2 * D + 3
    return g(h, u64) * T + u64 * (u32 * grow * A + (1 + g(h, u64)) * T)
