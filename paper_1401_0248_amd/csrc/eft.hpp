// eft.hpp: device-side error-free transforms and pair combines for gfx950.
//
// The per-element steps of the paper (Latkin, "Twofold fast summation",
// section "Algorithms"): Example 1 (fast twofold, Dekker's Theorem 1),
// Example 3 (rigorous twofold, Knuth's Theorem 2) and direct summation, with
// dot products by substitution of the product for the data item; this
// library adds the product's FMA remainder to the error. Compiled with
// -ffp-contract=off: the single FMA below is the only fused operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace twofold {

// kKahan: Example 2; kFastRounded / kRigorousRounded: the paper's own dot
// rule (the rounded product is the item; its rounding is not tracked).
// kWide is the paper's wider accumulator: for binary32 data a binary64 sum
// (kWide itself); for binary64 data, where the paper used quad precision,
// a double-word (double-double) sum, kDoubleDouble (internal only: the
// public mode is TWOFOLD_WIDE for both data types).
// kMixed (binary32 data only): the rigorous form with its error term in
// binary64. The value chain is the binary32 rigorous one; each step's exact
// round-off (and a dot's product remainder), binary32 numbers, are added to
// a binary64 error. Both parts live in binary64 registers, the value always
// holding a binary32 number.
enum Mode : int {
  kPlain = 0,
  kFast = 1,
  kRigorous = 2,
  kWide = 3,
  kKahan = 4,
  kFastRounded = 5,
  kRigorousRounded = 6,
  kMixed = 7,
  kDoubleDouble = 8,
  // Instrument only (the read probe): the "step" ORs the bits of the loaded
  // binary32 words into s, so the reductions' own load loop runs with no
  // arithmetic to wait for.
  kProbeOr = 9
};

// Modes whose pairs carry an error (all but plain, wide and the probe).
constexpr bool has_error(int m) { return m != kPlain && m != kWide && m != kProbeOr; }

// The combine used once block pairs are binary64 (step 7): a mixed pair's
// value is then a binary64 sum, combined like a rigorous pair.
constexpr int pass2_mode(int m) { return m == kMixed ? kRigorous : m; }

__device__ __forceinline__ float fma_rn(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_rn(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---- double-word arithmetic (kDoubleDouble) -------------------------------
// A double-word number is a pair (h, l) with h = fl(h + l). The additions
// are the published algorithms of Joldes, Muller and Popescu ("Tight and
// rigorous error bounds for basic building blocks of double-word
// arithmetic", ACM TOMS 2017): DWPlusFP (their Algorithm 4, relative error
// at most 2u^2) and AccurateDWPlusDW (their Algorithm 6, at most
// 3u^2 + 13u^3), built from two-sum (Theorem 2) and fast-two-sum (Theorem 1).
// Knuth's two-sum (Theorem 2): s = fl(a + b) and the exact remainder
// d = (a - av) + (b - bv), where bv = s - a and av = s - bv are the parts of
// s that came from b and from a; s + d = a + b for any finite a, b.
template <typename F>
__device__ __forceinline__ void two_sum(F a, F b, F& s, F& d) {
  s = a + b;
  const F bv = s - a;
  const F av = s - bv;
  d = (a - av) + (b - bv);
}

// Dekker's fast-two-sum (Theorem 1): s = fl(a + b), d = b - (s - a);
// s + d = a + b when |a| >= |b|.
template <typename F>
__device__ __forceinline__ void fast_two_sum(F a, F b, F& s, F& d) {
  s = a + b;
  d = b - (s - a);
}

// (h, l) += y
__device__ __forceinline__ void dw_add_fp(double& h, double& l, double y) {
  double sh, sl;
  two_sum(h, y, sh, sl);
  const double v = l + sl;
  fast_two_sum(sh, v, h, l);
}

// (h, l) += (yh, yl)
__device__ __forceinline__ void dw_add_dw(double& h, double& l, double yh, double yl) {
  double sh, sl, th, tl, vh, vl;
  two_sum(h, yh, sh, sl);
  two_sum(l, yl, th, tl);
  const double c = sl + th;
  fast_two_sum(sh, c, vh, vl);
  const double w = tl + vl;
  fast_two_sum(vh, w, h, l);
}

// One data item into one chain (s, e). T is the data type, A the
// accumulator type (A == T except in kWide, where binary32 data is widened
// to binary64 and summed plainly).
template <int M, bool DOT, typename T, typename A>
__device__ __forceinline__ void step(A& s, A& e, T xv, T yv) {
  if constexpr (M == kProbeOr) {
    static_assert(sizeof(T) == 4 && sizeof(A) == 4, "probe: binary32 words");
    uint32_t b = __float_as_uint(s) | __float_as_uint(xv);
    if constexpr (DOT) b |= __float_as_uint(yv);
    s = __uint_as_float(b);
  } else if constexpr (M == kWide) {
    A item = DOT ? static_cast<A>(xv) * static_cast<A>(yv) : static_cast<A>(xv);
    s = s + item;
  } else if constexpr (M == kDoubleDouble) {
    // (s, e) is the double-word accumulator; a dot adds the exact product
    // p + pi as a double-word number.
    if constexpr (DOT) {
      const double p = xv * yv;
      dw_add_dw(s, e, p, fma_rn(xv, yv, -p));
    } else {
      dw_add_fp(s, e, xv);
    }
  } else if constexpr (M == kMixed) {
    // the rigorous step in binary32 on the value; its exact remainder and
    // the product's join the binary64 error
    static_assert(sizeof(T) == 4 && sizeof(A) == 8, "mixed: binary32 data, binary64 registers");
    const float p = DOT ? xv * yv : xv;
    float t, r;
    two_sum(static_cast<float>(s), p, t, r);  // s holds a binary32 number: exact
    if constexpr (DOT) {
      e = e + (static_cast<double>(r) + static_cast<double>(fma_rn(xv, yv, -p)));
    } else {
      e = e + static_cast<double>(r);
    }
    s = static_cast<double>(t);
  } else if constexpr (M == kPlain) {
    T item = DOT ? xv * yv : xv;
    s = s + item;
  } else if constexpr (M == kKahan) {
    // Example 2 with e holding the negated correction: the item corrected
    // by e, then fast-two-sum of the value and the corrected item, whose
    // remainder is the next negated correction.
    const T item = DOT ? xv * yv : xv;
    fast_two_sum(s, item + e, s, e);
  } else {
    // The twofold steps: the value takes the item (a dot's rounded product
    // p); the error takes the step's remainder, from fast-two-sum (fast
    // form, Example 1: exact when |s| >= |item|) or two-sum (rigorous form,
    // Example 3: exact always), and for a dot with the exact product also
    // the product's FMA remainder x*y - p.
    constexpr bool kTrack = DOT && (M == kFast || M == kRigorous);
    constexpr bool kFastForm = (M == kFast || M == kFastRounded);
    const T p = DOT ? xv * yv : xv;
    T t, r;
    if constexpr (kFastForm) {
      fast_two_sum(s, p, t, r);
    } else {
      two_sum(s, p, t, r);
    }
    if constexpr (kTrack) {
      e = e + (r + fma_rn(xv, yv, -p));
    } else {
      e = e + r;
    }
    s = t;
  }
}

// combine((s1,e1),(s2,e2)): two-sum of the values with all six operations
// of Theorem 2, then the errors and the two-sum remainder. Plain and wide
// pairs carry no error; double-word pairs are added with AccurateDWPlusDW.
template <int M, typename A>
__device__ __forceinline__ void combine(A& s1, A& e1, A s2, A e2) {
  if constexpr (M == kProbeOr) {
    s1 = __uint_as_float(__float_as_uint(s1) | __float_as_uint(s2));
    e1 = A(0);
  } else if constexpr (!has_error(M)) {
    s1 = s1 + s2;
    e1 = A(0);
  } else if constexpr (M == kDoubleDouble) {
    dw_add_dw(s1, e1, s2, e2);  // double-word pairs add as double-word numbers
  } else if constexpr (M == kMixed) {
    // two-sum of the binary32 values in binary32, remainder into the
    // binary64 error
    float x, y;
    two_sum(static_cast<float>(s1), static_cast<float>(s2), x, y);
    e1 = (e1 + e2) + static_cast<double>(y);
    s1 = static_cast<double>(x);
  } else {
    A x, y;
    two_sum(s1, s2, x, y);
    e1 = (e1 + e2) + y;
    s1 = x;
  }
}

// ---- wave combine ---------------------------------------------------------
// Lane l receives the value of lane l - D: within its row of 16 lanes for
// D = 1, 2, 4, 8 (DPP row_shr), from lane 15 of the row before for D = 16
// (row_bcast:15, rows 1 and 3 written) and from lane 31 for D = 32
// (row_bcast:31, rows 2 and 3 written). Only the top lane of each group of
// 2D lanes uses the value, and for it the source lane is always valid. All
// moves are VALU data-parallel operations: no LDS access, so nothing waits
// on the LDS/scalar-memory counter.
template <int D>
__device__ __forceinline__ int from_lower_b32(int v) {
  if constexpr (D <= 8) {
    return __builtin_amdgcn_mov_dpp(v, 0x110 + D, 0xF, 0xF, false);
  } else if constexpr (D == 16) {
    return __builtin_amdgcn_mov_dpp(v, 0x142, 0xA, 0xF, false);
  } else {
    static_assert(D == 32, "distance");
    return __builtin_amdgcn_mov_dpp(v, 0x143, 0xC, 0xF, false);
  }
}

template <int D>
__device__ __forceinline__ float from_lower(float v) {
  return __int_as_float(from_lower_b32<D>(__float_as_int(v)));
}

template <int D>
__device__ __forceinline__ double from_lower(double v) {
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
  const int lo = from_lower_b32<D>(static_cast<int>(static_cast<uint32_t>(u)));
  const int hi = from_lower_b32<D>(static_cast<int>(static_cast<uint32_t>(u >> 32)));
  const uint64_t r = (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                     static_cast<uint64_t>(static_cast<uint32_t>(lo));
  return __longlong_as_double(static_cast<long long>(r));
}

// The top lane of each group of 2D lanes replaces its pair by
// combine(pair of lane l - D, own pair): the lower group's pair first.
template <int M, int D, typename A>
__device__ __forceinline__ void wave_stage(A& s, A& e) {
  A ls = from_lower<D>(s);
  A le = has_error(M) ? from_lower<D>(e) : A(0);
  combine<M>(ls, le, s, e);
  s = ls;
  e = le;
}

// The lane that holds a wave's combined pair.
constexpr int kWaveRoot = 63;

// Wave combine (step 5): distances 1, 2, 4, 8, 16, 32 in this order. After
// the stage of distance D the top lane of each aligned group of 2D lanes
// holds combine(lower D lanes, upper D lanes), each half combined the same
// way, so lane kWaveRoot ends with the pair that lane 0 holds after the
// documented exchange (where lane l combines its pair with lane l xor D's,
// its own first): both are the balanced binary tree over lanes 0..63 with
// the lower half's pair first in every combine. All 64 lanes must be active.
template <int M, typename A>
__device__ __forceinline__ void wave_combine(A& s, A& e) {
  wave_stage<M, 1>(s, e);
  wave_stage<M, 2>(s, e);
  wave_stage<M, 4>(s, e);
  wave_stage<M, 8>(s, e);
  wave_stage<M, 16>(s, e);
  wave_stage<M, 32>(s, e);
}

}  // namespace twofold
