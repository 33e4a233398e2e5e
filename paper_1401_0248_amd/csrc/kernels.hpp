// kernels.hpp: the twofold reduction kernels for gfx950.
//
// Streaming reductions bound by HBM bandwidth: 16-byte vector loads
// (global_load_dwordx4), U independent loads in flight per lane, W = 16 /
// sizeof(T) independent (s, e) chains per lane, then pair combines across
// chains, lanes (DPP), waves (LDS) and blocks
// (binary64, in one fixed order). No matrix cores: there is no contraction
// to feed them. The order is the one documented in include/twofold.h; it
// depends only on the launch configuration and the inputs, so results are
// identical run to run.
#pragma once

#include "eft.hpp"

namespace twofold {

constexpr int kPass2Lanes = 256;  // lanes of the binary64 grid combine

// Register budget. A kernel that may run blocks of 1024 threads must fit 16
// waves on a CU, four on each SIMD, and so gets at most 128 VGPRs a lane;
// one that runs blocks of at most 512 threads needs two waves a SIMD and
// may use 256. Each streaming kernel is built in both sizes (template
// parameter BMAX, its __launch_bounds__) and the host picks the instance
// from the launch's block size.
//
// Whether a lane keeps a second round of loads in flight while it works on
// the current one depends on what fits: two rounds of R = U*(1 + dot)
// 16-byte vectors take 8R VGPRs. Under the narrow budget that leaves room
// for R <= 4; under the wide one for R <= 8, i.e. every width but eight-
// vector dots, whose 128 VGPRs of buffers fit beside the rest of the
// single-vector kernel (216-253 VGPRs, no spill) but not beside the larger
// state of the multi-vector, batch and segmented kernels.
constexpr int kSmallBlock = 512;

template <int BMAX, bool DOT, int U>
constexpr bool rounds_ahead() {
  return U * (DOT ? 2 : 1) <= (BMAX <= kSmallBlock ? 8 : 4);
}

template <int BMAX, bool DOT, int U>
constexpr bool rounds_ahead_single() {
  return BMAX <= kSmallBlock || rounds_ahead<BMAX, DOT, U>();
}

template <typename T> struct vec16;
template <> struct vec16<float> { using type = float4; };
template <> struct vec16<double> { using type = double2; };

template <typename T>
__device__ __forceinline__ T vget(const typename vec16<T>::type& v, int j);
template <>
__device__ __forceinline__ float vget<float>(const float4& v, int j) {
  return j == 0 ? v.x : j == 1 ? v.y : j == 2 ? v.z : v.w;
}
template <>
__device__ __forceinline__ double vget<double>(const double2& v, int j) {
  return j == 0 ? v.x : v.y;
}

// Streaming loads: every input element is read exactly once, so all data
// loads carry the non-temporal hint (global_load ... nt). Measured on
// MI355X, a 1 GiB stream of 16-byte loads runs at about 7.1 TB/s with the
// hint against 6.5 TB/s without it.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ T load_nt(const T* p) {
  return __builtin_nontemporal_load(p);
}

// Load W consecutive elements starting at p + k*W. With ALIGNED the
// address is 16-byte aligned and one vector load is used; otherwise the
// elements are loaded one by one (same values, same order of use).
template <typename T, bool ALIGNED>
__device__ __forceinline__ typename vec16<T>::type load_vec(const T* __restrict__ p, int64_t k) {
  using V = typename vec16<T>::type;
  const T* q = p + k * (16 / static_cast<int64_t>(sizeof(T)));
  V v;
  if constexpr (ALIGNED) {
    if constexpr (sizeof(T) == 4) {
      const f32x4_t r = __builtin_nontemporal_load(reinterpret_cast<const f32x4_t*>(q));
      v.x = r.x;
      v.y = r.y;
      v.z = r.z;
      v.w = r.w;
    } else {
      const f64x2_t r = __builtin_nontemporal_load(reinterpret_cast<const f64x2_t*>(q));
      v.x = r.x;
      v.y = r.y;
    }
  } else {
    if constexpr (sizeof(T) == 4) {
      v.x = load_nt(q);
      v.y = load_nt(q + 1);
      v.z = load_nt(q + 2);
      v.w = load_nt(q + 3);
    } else {
      v.x = load_nt(q);
      v.y = load_nt(q + 1);
    }
  }
  return v;
}

// Elements before the first 16-byte boundary at or after p, capped at len.
template <typename T>
__device__ __forceinline__ int64_t head_count(const T* p, int64_t len) {
  const int64_t mis = static_cast<int64_t>(reinterpret_cast<uintptr_t>(p) & 15u) /
                      static_cast<int64_t>(sizeof(T));
  const int64_t W = 16 / static_cast<int64_t>(sizeof(T));
  const int64_t h = (W - mis) % W;
  return h < len ? h : len;
}

// v, hidden from the compiler's uniformity analysis. A head element is
// loaded by the lanes below the head count, which for binary64 data is at
// most 1: the compiler then proves the address uniform and makes the load a
// scalar one, waited for at once inside its branch, so the loads after it
// (tail, first round) wait a whole memory round trip before they are even
// issued. Indexed through this value it stays a vector load, waited for
// with the rest.
__device__ __forceinline__ int64_t opaque_lane(int64_t v) {
  asm("" : "+v"(v));
  return v;
}

// Steps 1-4 of the documented order for one lane g of L lanes over the
// range [x, x + len): head, rounds of U vectors, tail, chain merge.
//
// The head and tail elements are requested first. With AHEAD (see
// rounds_ahead) the loads also run one round ahead of the arithmetic: round
// 0 is requested with the head and tail, and while the steps of round q
// run, the loads of round q + 1 (or of the last, partial round) are in
// flight. Without it each round is loaded when it starts. Either way the
// steps are applied in the documented order (head, rounds in order, partial
// round, tail), so the result does not depend on when the data arrived.
template <typename T, typename A, int M, bool DOT, bool YV, int U, bool AHEAD>
__device__ __forceinline__ void lane_reduce(const T* __restrict__ x, const T* __restrict__ y,
                                            int64_t len, int64_t head, int64_t L, int64_t g,
                                            A& s_out, A& e_out) {
  constexpr int W = 16 / static_cast<int>(sizeof(T));
  constexpr bool kAhead = AHEAD;
  using V = typename vec16<T>::type;
  A cs[W], ce[W];
#pragma unroll
  for (int j = 0; j < W; j++) {
    cs[j] = A(0);
    ce[j] = A(0);
  }
  const T* __restrict__ xb = x + head;
  const T* __restrict__ yb = DOT ? y + head : nullptr;
  const int64_t nv = (len - head) / W;
  const int64_t tail0 = nv * W;
  const int64_t gh = opaque_lane(g);
  const bool has_head = gh < head;
  const bool has_tail = g < (len - head) - tail0;
  T hx = T(0), hy = T(0), tx = T(0), ty = T(0);
  if (has_head) {
    hx = load_nt(x + gh);
    if constexpr (DOT) hy = load_nt(y + gh);
  }
  if (has_tail) {
    tx = load_nt(xb + tail0 + g);
    if constexpr (DOT) ty = load_nt(yb + tail0 + g);
  }
  const int64_t per_round = static_cast<int64_t>(U) * L;
  const int64_t full = nv / per_round;
  // Round loads: all U vectors (full round) or those below nv (last round).
  auto load_round = [&](V (&a)[U], V (&b)[U], int64_t k, bool whole) {
    if (whole) {
#pragma unroll
      for (int u = 0; u < U; u++) a[u] = load_vec<T, true>(xb, k + u * L);
      if constexpr (DOT) {
#pragma unroll
        for (int u = 0; u < U; u++) b[u] = load_vec<T, YV>(yb, k + u * L);
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (k + u * L < nv) {
          a[u] = load_vec<T, true>(xb, k + u * L);
          if constexpr (DOT) b[u] = load_vec<T, YV>(yb, k + u * L);
        }
      }
    }
  };
  // Round steps, u in order: all U vectors (full round) or those below nv
  // (last round).
  auto step_round = [&](const V (&a)[U], const V (&b)[U], int64_t k, bool whole) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (whole || k + u * L < nv) {
#pragma unroll
        for (int j = 0; j < W; j++)
          step<M, DOT>(cs[j], ce[j], vget<T>(a[u], j), DOT ? vget<T>(b[u], j) : T(0));
      }
    }
  };
  int64_t k0 = g;
  if constexpr (kAhead) {
    // Two round buffers used in turn (a0/b0, a1/b1), so that no register
    // is copied while its load may still be in flight: the loads of round
    // q + 1 stay outstanding while the steps of round q run.
    V a0[U], b0[U], a1[U], b1[U];
    if (full == 0) {
      load_round(a0, b0, k0, false);
      if (has_head) step<M, DOT>(cs[0], ce[0], hx, hy);
      step_round(a0, b0, k0, false);  // the partial round alone
    } else {
      load_round(a0, b0, k0, true);
      if (has_head) step<M, DOT>(cs[0], ce[0], hx, hy);
      // a0/b0 holds full round q on entry; rounds q + 1 and q + 2 are full
      int64_t q = 0;
      for (; q + 2 < full; q += 2) {
        load_round(a1, b1, k0 + per_round, true);
        step_round(a0, b0, k0, true);
        k0 += per_round;
        load_round(a0, b0, k0 + per_round, true);
        step_round(a1, b1, k0, true);
        k0 += per_round;
      }
      if (q + 1 < full) {  // two full rounds left, then the partial one
        load_round(a1, b1, k0 + per_round, true);
        step_round(a0, b0, k0, true);
        k0 += per_round;
        load_round(a0, b0, k0 + per_round, false);
        step_round(a1, b1, k0, true);
        k0 += per_round;
        step_round(a0, b0, k0, false);
      } else {  // one full round left, then the partial one
        load_round(a1, b1, k0 + per_round, false);
        step_round(a0, b0, k0, true);
        k0 += per_round;
        step_round(a1, b1, k0, false);
      }
    }
  } else {
    if (has_head) step<M, DOT>(cs[0], ce[0], hx, hy);
    for (int64_t q = 0; q < full; q++, k0 += per_round) {
      V a[U], b[U];
      load_round(a, b, k0, true);
      step_round(a, b, k0, true);
    }
    V a[U], b[U];
    load_round(a, b, k0, false);
    step_round(a, b, k0, false);  // last, partial round
  }
  if (has_tail) step<M, DOT>(cs[0], ce[0], tx, ty);
  A s = cs[0], e = ce[0];
#pragma unroll
  for (int j = 1; j < W; j++) combine<M>(s, e, cs[j], ce[j]);
  s_out = s;
  e_out = e;
}

// Step 8: binary64 (V, E) into the output pair.
template <typename T, int M>
__device__ __forceinline__ void finalize_store(void* __restrict__ out, int64_t idx, double V,
                                               double E) {
  if constexpr (sizeof(T) == 8 || M == kWide) {
    reinterpret_cast<double2*>(out)[idx] = make_double2(V, E);
  } else if constexpr (M == kMixed) {
    // value fl32(V), error (V - value) + E in binary64 (V - value is exact)
    const double v = static_cast<double>(static_cast<float>(V));
    reinterpret_cast<double2*>(out)[idx] = make_double2(v, (V - v) + E);
  } else {
    const float v = static_cast<float>(V);
    float e = 0.0f;
    if constexpr (has_error(M)) e = static_cast<float>((V - static_cast<double>(v)) + E);
    reinterpret_cast<float2*>(out)[idx] = make_float2(v, e);
  }
}

__device__ __forceinline__ void store_nan_pair(void* out, int64_t idx, bool f64_pair) {
  if (f64_pair)
    reinterpret_cast<double2*>(out)[idx] = make_double2(__builtin_nan(""), __builtin_nan(""));
  else
    reinterpret_cast<float2*>(out)[idx] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
}

template <typename T, int M>
constexpr bool out_is_f64() {
  return sizeof(T) == 8 || M == kWide || M == kMixed;
}

// ---- single vector ----------------------------------------------------------
// Pass 1: one pair per block. With one block the pair is final (steps 7-8);
// otherwise it goes to part[] in binary64 and pass 2 combines the block
// pairs in index order. The two passes are separate kernels: the kernel
// boundary orders them, so no block ever waits on, or fences for, another.
// Steps 5-6 for the lane pairs (s, e) of one vector: the block pair goes to
// part[blockIdx.x], or, with one block, finalized to out[idx].
template <typename T, typename A, int M>
__device__ __forceinline__ void block_store(A s, A e, double* __restrict__ part,
                                            void* __restrict__ out, int64_t idx) {
  __shared__ A sh_s[16], sh_e[16];
  wave_combine<M>(s, e);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  if (lane == kWaveRoot) {
    sh_s[wave] = s;
    sh_e[wave] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    A bs = sh_s[0], be = sh_e[0];
    for (int w = 1; w < nw; w++) combine<M>(bs, be, sh_s[w], sh_e[w]);
    if (gridDim.x == 1) {
      finalize_store<T, M>(out, idx, static_cast<double>(bs), static_cast<double>(be));
    } else {
      reinterpret_cast<double2*>(part)[blockIdx.x] =
          make_double2(static_cast<double>(bs), static_cast<double>(be));
    }
  }
}

// Steps 1-6 for block blockIdx.x of a grid of gridDim.x blocks over one
// vector.
template <typename T, typename A, int M, bool DOT, bool YV, int U, bool AHEAD>
__device__ __forceinline__ void single_block(const T* __restrict__ x, const T* __restrict__ y,
                                             int64_t n, double* __restrict__ part,
                                             void* __restrict__ out, int64_t idx) {
  const int64_t L = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t head = head_count(x, n);
  A s, e;
  lane_reduce<T, A, M, DOT, YV, U, AHEAD>(x, y, n, head, L, g, s, e);
  block_store<T, A, M>(s, e, part, out, idx);
}

template <typename T, typename A, int M, bool DOT, bool YV, int U, int BMAX>
__global__ void __launch_bounds__(BMAX)
single_kernel(const T* __restrict__ x, const T* __restrict__ y, int64_t n,
              double* __restrict__ part, void* __restrict__ out) {
  single_block<T, A, M, DOT, YV, U, rounds_ahead_single<BMAX, DOT, U>()>(x, y, n, part, out, 0);
}

// ---- several vectors in one launch ------------------------------------------
// A multi-vector launch has gridDim.y sets of gridDim.x blocks. Set r takes
// vectors r, r + gridDim.y, ... in turn, and its block b reduces its share
// of vector v exactly as block b of a single-vector call with the same
// launch does (steps 1-6; the block pairs of vector v at
// part[v * gridDim.x ...]). One set walking all the vectors streams them
// like one long vector; one set per vector runs short vectors side by side.
// Either way every pair is the same. The addresses and lengths travel in
// the kernel arguments.
constexpr int kMaxMulti = 64;

template <typename T>
struct MultiArgs {
  const T* x[kMaxMulti];
  const T* y[kMaxMulti];
  int64_t n[kMaxMulti];
};

template <typename T, typename A, int M, bool DOT, bool YV, int U, int BMAX>
__global__ void __launch_bounds__(BMAX)
multi_kernel(const MultiArgs<T> args, int count, double* __restrict__ part,
             void* __restrict__ out) {
  for (int v = blockIdx.y; v < count; v += gridDim.y) {
    single_block<T, A, M, DOT, YV, U, rounds_ahead<BMAX, DOT, U>()>(args.x[v], args.y[v], args.n[v],
                                      part + 2 * static_cast<int64_t>(v) * gridDim.x, out, v);
    __syncthreads();  // the block combine's LDS is reused for the next vector
  }
}

// Lane l of a combine over `stride` lanes: pairs l, l + stride, ... of
// p[0 .. count), combined into (qs, qe) in that order (from +0). The loads run
// up to eight pairs ahead of the combines, which stay in order.
template <int M>
__device__ __forceinline__ void combine_strided(const double2* __restrict__ p, int64_t count,
                                                int64_t l, int64_t stride, double& qs, double& qe) {
  constexpr int kAhead = 8;
  for (int64_t i0 = l; i0 < count; i0 += kAhead * stride) {
    double2 v[kAhead];
#pragma unroll
    for (int k = 0; k < kAhead; k++)
      if (i0 + k * stride < count) v[k] = p[i0 + k * stride];
#pragma unroll
    for (int k = 0; k < kAhead; k++)
      if (i0 + k * stride < count) combine<M>(qs, qe, v[k].x, v[k].y);
  }
}

// Pass 2 (step 7): block b of kPass2Lanes threads combines the nparts block
// pairs of vector b (part[b * nparts ...]; one block for a single-vector
// call) in binary64, lane l taking pairs l, l + 256, ... in order.
template <typename T, int M>
__device__ __forceinline__ void pass2_block(const double2* __restrict__ pairs, int nparts,
                                            void* __restrict__ out, int64_t idx) {
  __shared__ double sh_s[kPass2Lanes / 64], sh_e[kPass2Lanes / 64];
  constexpr int P = pass2_mode(M);
  double qs = 0.0, qe = 0.0;
  combine_strided<P>(pairs, nparts, threadIdx.x, kPass2Lanes, qs, qe);
  wave_combine<P>(qs, qe);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == kWaveRoot) {
    sh_s[wave] = qs;
    sh_e[wave] = qe;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double V = sh_s[0], E = sh_e[0];
    for (int w = 1; w < kPass2Lanes / 64; w++) combine<P>(V, E, sh_s[w], sh_e[w]);
    finalize_store<T, M>(out, idx, V, E);
  }
}

template <typename T, int M>
__global__ void __launch_bounds__(kPass2Lanes)
single_pass2_kernel(const double* __restrict__ part, int nparts, void* __restrict__ out) {
  pass2_block<T, M>(reinterpret_cast<const double2*>(part) + static_cast<int64_t>(blockIdx.x) * nparts,
                    nparts, out, blockIdx.x);
}

// ---- segmented ---------------------------------------------------------------

// One wave's walk over its tiles. Segment sg covers tiles [tb, tend) and
// elements [oa, ob); these stay in (scalar) registers while the wave walks
// the segment's tiles, and the next segment's bounds are requested as soon
// as a segment is entered, so moving on to it does not wait for memory.
struct SegWalk {
  const int64_t* __restrict__ off;
  const int64_t* __restrict__ tbase;
  int64_t nseg, TS, sg;
  int64_t tb = 0, tend = 0, oa = 0, ob = 0, nx_tend = 0, nx_ob = 0;

  __device__ __forceinline__ void prefetch() {
    if (sg + 1 != nseg) {  // sg < nseg
      nx_tend = tbase[sg + 2];
      nx_ob = off[sg + 2];
    }
  }
  // Enter the segment of tile t (sg at or before it).
  __device__ __forceinline__ void start(int64_t t) {
    while (tbase[sg + 1] <= t) sg++;
    tb = tbase[sg];
    tend = tbase[sg + 1];
    oa = off[sg];
    ob = off[sg + 1];
    prefetch();
  }
  // Move on to tile t: the current one or the next (t <= tend, so the
  // tests are equalities, which the scalar unit does on 64 bits).
  __device__ __forceinline__ void to(int64_t t) {
    if (t != tend) return;
    sg++;
    tb = tend;
    oa = ob;
    tend = nx_tend;
    ob = nx_ob;
    while (tend == t) {  // empty segments in between
      sg++;
      tb = tend;
      oa = ob;
      tend = tbase[sg + 1];
      ob = off[sg + 1];
    }
    prefetch();
  }
  __device__ __forceinline__ int64_t begin(int64_t t) const { return oa + (t - tb) * TS; }
  __device__ __forceinline__ int64_t end(int64_t t) const {
    const int64_t a = begin(t);
    return ob < a + TS ? ob : a + TS;
  }
};

// Steps 5 and the store of one tile's pair: a one-tile segment's pair is
// finalized (step 8), a longer segment's goes to its tile slot.
template <typename T, typename A, int M>
__device__ __forceinline__ void tile_store(A s, A e, int lane, int64_t t, int64_t sg, int64_t ntl,
                                           double* __restrict__ slots, void* __restrict__ out) {
  wave_combine<M>(s, e);
  if (lane == kWaveRoot) {
    if (ntl == 1)
      finalize_store<T, M>(out, sg, static_cast<double>(s), static_cast<double>(e));
    else
      reinterpret_cast<double2*>(slots)[t] =
          make_double2(static_cast<double>(s), static_cast<double>(e));
  }
}

// The tiles [t0, t1) of one wave with loads one round ahead of the steps,
// across tile boundaries too: the next tile's head, tail and first round
// are requested before the current tile's last (partial) round, tail and
// combine. (The compiler waits for them where they move into the round
// buffers at the next tile's start, so at a tile boundary no other load is
// in flight; a variant without that move was no faster.) Per tile, the
// steps are those of lane_reduce with L = 64, in the same order, so every
// pair is the same.
template <typename T, typename A, int M, bool DOT, bool YV, int U>
__device__ __forceinline__ void seg_tiles_ahead(const T* __restrict__ x, const T* __restrict__ y,
                                                SegWalk& wk, int64_t t0, int64_t t1, int lane,
                                                double* __restrict__ slots, void* __restrict__ out) {
  constexpr int W = 16 / static_cast<int>(sizeof(T));
  constexpr int64_t PR = static_cast<int64_t>(U) * 64;  // vectors per round
  using V = typename vec16<T>::type;
  // The geometry of a tile [a, a + len): head elements, body vectors, full
  // rounds (uniform across the wave).
  // A tile holds at most TS <= 2^30 elements, so everything but its start
  // is 32-bit: the tests on it are scalar compares. (A 64-bit ordered
  // compare of scalars goes through a vector register, which the compiler
  // may take from a round buffer with loads in flight and wait for them.)
  struct Geo {
    int64_t a;
    int32_t len, head, nv, full;
  };
  auto geo = [&](int64_t t) {
    Geo g;
    g.a = wk.begin(t);
    // every tile of a segment but its last holds TS elements
    g.len = (t + 1 != wk.tend) ? static_cast<int32_t>(wk.TS) : static_cast<int32_t>(wk.ob - g.a);
    const int32_t mis = static_cast<int32_t>(reinterpret_cast<uintptr_t>(x + g.a) & 15u) /
                        static_cast<int32_t>(sizeof(T));
    const int32_t h = (W - mis) % W;
    g.head = h < g.len ? h : g.len;
    g.nv = (g.len - g.head) / W;
    g.full = g.nv / static_cast<int32_t>(PR);
    return g;
  };
  // A tile's first loads: head and tail elements, then round 0 (or, with no
  // full round, the vectors of the partial round).
  auto first_loads = [&](const Geo& g, V (&va)[U], V (&vb)[U], T& hx, T& hy, T& tx, T& ty) {
    const T* xa = x + g.a;
    const T* ya = DOT ? y + g.a : nullptr;
    const T* xb = xa + g.head;
    const T* yb = DOT ? ya + g.head : nullptr;
    const int64_t tail0 = static_cast<int64_t>(g.nv) * W;
    hx = hy = tx = ty = T(0);
    const int64_t hl = opaque_lane(lane);
    if (hl < g.head) {
      hx = load_nt(xa + hl);
      if constexpr (DOT) hy = load_nt(ya + hl);
    }
    if (lane < (g.len - g.head) - g.nv * W) {
      tx = load_nt(xb + tail0 + lane);
      if constexpr (DOT) ty = load_nt(yb + tail0 + lane);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t k = lane + u * 64;
      if (g.full > 0 || k < g.nv) {
        va[u] = load_vec<T, true>(xb, k);
        if constexpr (DOT) vb[u] = load_vec<T, YV>(yb, k);
      }
    }
  };
  Geo g = geo(t0);
  V va[U], vb[U];
  T hx, hy, tx, ty;
  first_loads(g, va, vb, hx, hy, tx, ty);
  // (t0 < t1; tests of tile indices as equalities, see SegWalk::to)
  for (int64_t t = t0; t != t1; t++) {
    const int64_t sg = wk.sg, ntl = wk.tend - wk.tb;
    const T* xb = x + g.a + g.head;
    const T* yb = DOT ? y + g.a + g.head : nullptr;
    A cs[W], ce[W];
#pragma unroll
    for (int j = 0; j < W; j++) {
      cs[j] = A(0);
      ce[j] = A(0);
    }
    if (lane < g.head) step<M, DOT>(cs[0], ce[0], hx, hy);
    // Rounds in turn through va/vb and na/nb: the loads of the next round
    // are issued before the steps of the current one and no round is copied
    // while in flight. A tile with an odd number of full rounds ends with
    // its partial round in na/nb, which is then moved to va/vb once.
    int64_t k0 = lane;
    V na[U], nb[U];
    auto load_into = [&](V (&a)[U], V (&b)[U], int64_t k, bool whole) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (whole || k + u * 64 < g.nv) {
          a[u] = load_vec<T, true>(xb, k + u * 64);
          if constexpr (DOT) b[u] = load_vec<T, YV>(yb, k + u * 64);
        }
      }
    };
    auto step_full = [&](const V (&a)[U], const V (&b)[U]) {
#pragma unroll
      for (int u = 0; u < U; u++) {
#pragma unroll
        for (int j = 0; j < W; j++)
          step<M, DOT>(cs[j], ce[j], vget<T>(a[u], j), DOT ? vget<T>(b[u], j) : T(0));
      }
    };
    // (only whole rounds inside the loop, so its loads carry no condition
    // and the waits count exactly)
    int32_t q = 0;
    for (; q + 2 < g.full; q += 2) {  // va holds full round q; rounds q + 1, q + 2 are full
      load_into(na, nb, k0 + PR, true);
      step_full(va, vb);
      k0 += PR;
      load_into(va, vb, k0 + PR, true);
      step_full(na, nb);
      k0 += PR;
    }
    if (q + 1 < g.full) {  // two full rounds left
      load_into(na, nb, k0 + PR, true);
      step_full(va, vb);
      k0 += PR;
      load_into(va, vb, k0 + PR, false);
      step_full(na, nb);
      k0 += PR;
    } else if (q < g.full) {  // one full round left
      load_into(na, nb, k0 + PR, false);
      step_full(va, vb);
      k0 += PR;
#pragma unroll
      for (int u = 0; u < U; u++) {
        va[u] = na[u];
        if constexpr (DOT) vb[u] = nb[u];
      }
    }
    // The next tile's first loads go out before this tile's last round.
    Geo gn = g;
    V wa[U], wb[U];
    T nhx = T(0), nhy = T(0), ntx = T(0), nty = T(0);
    if (t + 1 != t1) {
      wk.to(t + 1);
      gn = geo(t + 1);
      first_loads(gn, wa, wb, nhx, nhy, ntx, nty);
    }
    // last, partial round, then the tail
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (k0 + u * 64 < g.nv) {
#pragma unroll
        for (int j = 0; j < W; j++)
          step<M, DOT>(cs[j], ce[j], vget<T>(va[u], j), DOT ? vget<T>(vb[u], j) : T(0));
      }
    }
    if (lane < (g.len - g.head) - g.nv * W) step<M, DOT>(cs[0], ce[0], tx, ty);
    A s = cs[0], e = ce[0];
#pragma unroll
    for (int j = 1; j < W; j++) combine<M>(s, e, cs[j], ce[j]);
    tile_store<T, A, M>(s, e, lane, t, sg, ntl, slots, out);
    g = gn;
#pragma unroll
    for (int u = 0; u < U; u++) {
      va[u] = wa[u];
      if constexpr (DOT) vb[u] = wb[u];
    }
    hx = nhx;
    hy = nhy;
    tx = ntx;
    ty = nty;
  }
}


// Which wave takes which tile does not change any result; the assignment
// balances time. A tile costs its length plus c0 elements, c0 standing for
// its start-up and finish (the first loads' round trip, the combine and the
// store): measured on MI355X as about as long as streaming 16 KiB of input,
// whatever the unroll (a sweep of c0 on batches of 20,000 log-uniform
// segments put the best balance at 12-32 KiB for both data types). So
// c0 = kSegTileCostBytes / (bytes of one element position), the tiles
// before segment s cost cbase(s) = (off[s] - off[0]) + c0*tbase[s], and the
// total is C = cbase(nseg). Wave w of NW takes the tiles whose start cost
// lies in [floor(w*C/NW), floor((w+1)*C/NW)).
constexpr int64_t kSegTileCostBytes = 16384;

constexpr int64_t seg_tile_cost(int64_t elem_bytes, bool dot) {
  return kSegTileCostBytes / (elem_bytes * (dot ? 2 : 1));
}
__device__ __forceinline__ int64_t seg_cost_bound(int64_t w, int64_t C, int64_t NW) {
  return static_cast<int64_t>((static_cast<__int128>(w) * C) / NW);
}

// Pass 1: persistent waves over the tile list. tbase[s] = number of tiles
// of the segments before s (tbase[nseg] = total NT). With a wave table
// (plans), wave w reads its first tile, that tile's segment and its end
// from wtab[2w], wtab[2w+1], wtab[2w+2]; without one it finds them by two
// interleaved binary searches over the segments' costs. A one-tile segment
// is finalized here; the pair of a tile of a longer segment goes to
// slots[tile].
template <typename T, typename A, int M, bool DOT, bool YV, int U, int BMAX>
__global__ void __launch_bounds__(BMAX)
seg_kernel(const T* __restrict__ x, const T* __restrict__ y, const int64_t* __restrict__ off,
           int64_t nseg, const int64_t* __restrict__ tbase, const int64_t* __restrict__ wtab,
           int64_t TS, const uint32_t* __restrict__ status, double* __restrict__ slots,
           void* __restrict__ out) {
  if (status && *status != 0) return;  // invalid offsets: pass 2 reports NaN
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6;
  // the wave's index, made visibly uniform so its tile walk and the
  // segment bounds below use scalar registers and scalar loads
  const int64_t w = static_cast<int64_t>(blockIdx.x) * wpb +
                    __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  int64_t t0, t1, sg;
  if (wtab) {
    t0 = wtab[2 * w];
    sg = wtab[2 * w + 1];
    t1 = wtab[2 * w + 2];
  } else {
    constexpr int64_t c0 = seg_tile_cost(sizeof(T), DOT);
    const int64_t NW = static_cast<int64_t>(gridDim.x) * wpb;
    const int64_t o0 = off[0];
    const int64_t C = (off[nseg] - o0) + c0 * tbase[nseg];
    const int64_t lo0 = seg_cost_bound(w, C, NW), lo1 = seg_cost_bound(w + 1, C, NW);
    // Largest segment a with cbase(a) <= lo (cbase(0) = 0 <= lo), for both
    // bounds at once.
    int64_t a0 = 0, a1 = 0, n = nseg;
    while (n > 1) {
      const int64_t half = n >> 1;
      const int64_t m0 = a0 + half, m1 = a1 + half;
      if ((off[m0] - o0) + c0 * tbase[m0] <= lo0) a0 = m0;
      if ((off[m1] - o0) + c0 * tbase[m1] <= lo1) a1 = m1;
      n -= half;
    }
    // First tile at or after each bound: tile i of segment a starts at cost
    // cbase(a) + i*(TS + c0); past the segment's last tile, the next
    // segment's first tile.
    const int64_t i0 = ((lo0 - (off[a0] - o0) - c0 * tbase[a0]) + TS + c0 - 1) / (TS + c0);
    const int64_t i1 = ((lo1 - (off[a1] - o0) - c0 * tbase[a1]) + TS + c0 - 1) / (TS + c0);
    t0 = (i0 < tbase[a0 + 1] - tbase[a0]) ? tbase[a0] + i0 : tbase[a0 + 1];
    t1 = (i1 < tbase[a1 + 1] - tbase[a1]) ? tbase[a1] + i1 : tbase[a1 + 1];
    sg = a0;
  }
  if (t0 >= t1) return;
  SegWalk wk{off, tbase, nseg, TS, sg};
  wk.start(t0);
  if constexpr (rounds_ahead<BMAX, DOT, U>()) {
    seg_tiles_ahead<T, A, M, DOT, YV, U>(x, y, wk, t0, t1, lane, slots, out);
  } else {
    // Tile by tile. Under the wide register budget (eight-vector dots: the
    // cross-tile walk would need a third round buffer) the binary32 forms
    // still keep their loads a round ahead inside each tile; the forms with
    // binary64 chains would spill doing so (12-36 bytes a lane), so they
    // load each round when it starts.
    constexpr bool kInTile = BMAX <= kSmallBlock && sizeof(A) == 4;
    for (int64_t t = t0; t < t1; t++) {
      wk.to(t);
      const int64_t a = wk.begin(t), b = wk.end(t);
      const T* xa = x + a;
      const T* ya = DOT ? y + a : nullptr;
      A s, e;
      lane_reduce<T, A, M, DOT, YV, U, kInTile>(xa, ya, b - a, head_count(xa, b - a), 64, lane, s,
                                                e);
      tile_store<T, A, M>(s, e, lane, t, wk.sg, wk.tend - wk.tb, slots, out);
    }
  }
}

// Pass 2: one wave per segment, the waves of the grid striding over the
// segments (so the grid stays small for any segment count). Empty segments
// get (+0, +0); segments of two or more tiles combine their tile pairs in
// binary64 (lane l takes tiles l, l + 64, ... in tile order), then the wave
// combine and step 8. With invalid offsets (device-offset path) every
// output is NaN.
constexpr int kSegPass2Threads = 256;
constexpr int64_t kSegPass2MaxBlocks = 8192;

// Blocks of a pass-2 launch over nseg segments: one wave per segment up to
// kSegPass2MaxBlocks blocks, then the waves stride.
inline int64_t seg_pass2_blocks(int64_t nseg) {
  const int64_t wpb = kSegPass2Threads / 64;
  const int64_t b = (nseg + wpb - 1) / wpb;
  return b < 1 ? 1 : (b > kSegPass2MaxBlocks ? kSegPass2MaxBlocks : b);
}

template <typename T, int M>
__global__ void __launch_bounds__(kSegPass2Threads)
seg_pass2_kernel(const int64_t* __restrict__ tbase, int64_t nseg,
                 const uint32_t* __restrict__ status, const double* __restrict__ slots,
                 void* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t nw = static_cast<int64_t>(gridDim.x) * wpb;
  const bool bad = status && *status != 0;
  for (int64_t sg = static_cast<int64_t>(blockIdx.x) * wpb + (threadIdx.x >> 6); sg < nseg;
       sg += nw) {
    if (bad) {
      if (lane == 0) store_nan_pair(out, sg, out_is_f64<T, M>());
      continue;
    }
    const int64_t tb = tbase[sg];
    const int64_t ntl = tbase[sg + 1] - tb;
    if (ntl == 1) continue;
    if (ntl == 0) {
      if (lane == 0) finalize_store<T, M>(out, sg, 0.0, 0.0);
      continue;
    }
    constexpr int P = pass2_mode(M);
    double qs = 0.0, qe = 0.0;
    combine_strided<P>(reinterpret_cast<const double2*>(slots) + tb, ntl, lane, 64, qs, qe);
    wave_combine<P>(qs, qe);
    if (lane == kWaveRoot) finalize_store<T, M>(out, sg, qs, qe);
  }
}

}  // namespace twofold
