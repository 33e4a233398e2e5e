// segmented.hip: host side of the segmented (CSR batch) entry points of
// include/twofold.h: device-offset calls and plans.
//
// Device-offset calls run three kernels (tiling, tiles, per-segment
// combine); plan executes run the last two, with the tile table built once
// on the host. Nothing on an execute path allocates, frees or synchronises.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdlib.h>

#include "host_common.hpp"
#include "kernels.hpp"
#include "twofold.h"

using namespace twofold;
using namespace twofold::host;

namespace {

// Tile table and wave table from device offsets, in three kernels over
// rows of kSegRow segments (one block of kSegRow threads a row; the grids
// stride over rows).
//
// 1. Each segment's tiles, their exclusive scan within the row (in LDS,
//    into tbase), the row's total into rows[r] and whether the row's
//    offsets are invalid into bad[r] (offsets[0] >= 0, non-decreasing,
//    offsets[nseg] <= n_total).
__global__ void __launch_bounds__(kSegRow)
seg_count_kernel(const int64_t* __restrict__ off, int64_t nseg, int64_t n_total, int64_t TS,
                 int64_t* __restrict__ tbase, int64_t* __restrict__ rows,
                 uint32_t* __restrict__ bad) {
  __shared__ int64_t sh[kSegRow];
  const int t = threadIdx.x;
  const int64_t nrow = (nseg + kSegRow - 1) / kSegRow;
  for (int64_t r = blockIdx.x; r < nrow; r += gridDim.x) {
    const int64_t sg = r * kSegRow + t;
    int64_t tiles = 0;
    int b = 0;
    if (sg < nseg) {
      const int64_t len = off[sg + 1] - off[sg];
      b = len < 0;
      tiles = len > 0 ? (len + TS - 1) / TS : 0;
    }
    if (r == 0 && t == 0 && (off[0] < 0 || off[nseg] > n_total)) b = 1;
    sh[t] = tiles;
    __syncthreads();
    for (int d = 1; d < kSegRow; d <<= 1) {  // inclusive Hillis-Steele scan
      const int64_t v = t >= d ? sh[t - d] : 0;
      __syncthreads();
      sh[t] += v;
      __syncthreads();
    }
    if (sg < nseg) tbase[sg] = sh[t] - tiles;
    const int any = __syncthreads_or(b);
    if (t == 0) {
      rows[r] = sh[kSegRow - 1];
      bad[r] = any ? 1u : 0u;
    }
    __syncthreads();  // sh is reused by the next row
  }
}

// 2. (one block) The rows' totals become their exclusive prefix sums,
//    rows[nrow] the number of tiles, and *status whether any row is invalid.
__global__ void __launch_bounds__(kSegRow)
seg_rows_kernel(int64_t nrow, int64_t* __restrict__ rows, const uint32_t* __restrict__ bad,
                uint32_t* __restrict__ status) {
  __shared__ int64_t sh[kSegRow];
  const int t = threadIdx.x;
  int64_t carry = 0;
  int b = 0;
  for (int64_t base = 0; base < nrow; base += kSegRow) {
    const int64_t r = base + t;
    const int64_t v = r < nrow ? rows[r] : 0;
    if (r < nrow && bad[r]) b = 1;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < kSegRow; d <<= 1) {
      const int64_t u = t >= d ? sh[t - d] : 0;
      __syncthreads();
      sh[t] += u;
      __syncthreads();
    }
    if (r < nrow) rows[r] = carry + sh[t] - v;
    carry += sh[kSegRow - 1];
    __syncthreads();
  }
  const int any = __syncthreads_or(b);
  if (t == 0) {
    rows[nrow] = carry;
    *status = any ? 1u : 0u;
  }
}

// 3. Each segment's tile base gets its row's prefix, tbase[nseg] the number
//    of tiles; with valid offsets, the wave table of the launch (nw waves;
//    the cost model and meaning of a plan's, build_wave_table): segment s
//    covers the start costs [cbase(s), cbase(s + 1)) and writes the entries
//    of the waves w < nw whose bound floor(w*C/nw) falls there. With no
//    tiles at all every wave gets the empty range.
__global__ void __launch_bounds__(kSegRow)
seg_finish_kernel(const int64_t* __restrict__ off, int64_t nseg, int64_t TS, int64_t c0,
                  int64_t* __restrict__ tbase, const int64_t* __restrict__ rows,
                  const uint32_t* __restrict__ status, int64_t nw, int64_t* __restrict__ wtab) {
  const int t = threadIdx.x;
  const int64_t nrow = (nseg + kSegRow - 1) / kSegRow;
  const int64_t NT = rows[nrow];
  const bool table = wtab && *status == 0;
  const int64_t o0 = off[0];
  const int64_t C = table ? (off[nseg] - o0) + c0 * NT : 0;
  if (blockIdx.x == 0 && t == 0) {
    tbase[nseg] = NT;
    if (table) {
      wtab[2 * nw] = NT;
      wtab[2 * nw + 1] = nseg - 1;
    }
  }
  if (table && C == 0) {
    for (int64_t w = int64_t(blockIdx.x) * kSegRow + t; w < nw; w += int64_t(gridDim.x) * kSegRow) {
      wtab[2 * w] = 0;
      wtab[2 * w + 1] = 0;
    }
  }
  for (int64_t r = blockIdx.x; r < nrow; r += gridDim.x) {
    const int64_t sg = r * kSegRow + t;
    if (sg >= nseg) continue;
    const int64_t tb = tbase[sg] + rows[r];
    tbase[sg] = tb;
    if (!table || C == 0) continue;
    const int64_t len = off[sg + 1] - off[sg];
    const int64_t ntl = len > 0 ? (len + TS - 1) / TS : 0;
    const int64_t a = (off[sg] - o0) + c0 * tb;  // cbase(sg)
    const int64_t b = a + len + c0 * ntl;         // cbase(sg + 1)
    // the waves with a <= floor(w*C/nw) < b: w in [ceil(a*nw/C), ceil(b*nw/C))
    auto ceil_w = [&](int64_t c) {
      return static_cast<int64_t>((static_cast<__int128>(c) * nw + (C - 1)) / C);
    };
    const int64_t we = ceil_w(b) < nw ? ceil_w(b) : nw;
    for (int64_t w = ceil_w(a); w < we; w++) {
      const int64_t lo = static_cast<int64_t>((static_cast<__int128>(w) * C) / nw);
      const int64_t i = ((lo - a) + TS + c0 - 1) / (TS + c0);
      wtab[2 * w] = i < ntl ? tb + i : tb + ntl;
      wtab[2 * w + 1] = sg;
    }
  }
}

template <typename T, typename A, int M, bool DOT, bool YV>
int launch_seg_u(const T* x, const T* y, const int64_t* off, int64_t nseg, const int64_t* tbase,
                 const int64_t* wtab, const uint32_t* status, const twofold_launch_t& lc,
                 double* slots, void* out, hipStream_t st) {
  const dim3 grid(lc.grid_blocks), block(lc.block_threads);
  const int64_t ts = lc.tile_elems;
  const int rc = by_shape(lc, [&](auto u, auto bmax) {
    return launch_kernel(seg_kernel<T, A, M, DOT, YV, decltype(u)::value, decltype(bmax)::value>,
                         grid, block, st, x, y, off, nseg, tbase, wtab, ts, status, slots, out);
  });
  if (rc) return rc;
  return launch_kernel(seg_pass2_kernel<T, M>, dim3(unsigned(seg_pass2_blocks(nseg))),
                       dim3(kSegPass2Threads), st, tbase, nseg, status, slots, out);
}

template <typename T, typename A, int M, bool DOT>
int launch_seg(const T* x, const T* y, const int64_t* off, int64_t nseg, const int64_t* tbase,
               const int64_t* wtab, const uint32_t* status, const twofold_launch_t& lc,
               double* slots, void* out, hipStream_t st) {
  if constexpr (DOT) {
    if (!y_vector_ok(x, y))
      return launch_seg_u<T, A, M, DOT, false>(x, y, off, nseg, tbase, wtab, status, lc, slots,
                                               out, st);
  }
  return launch_seg_u<T, A, M, DOT, true>(x, y, off, nseg, tbase, wtab, status, lc, slots, out,
                                          st);
}

template <typename T, bool DOT>
int seg_by_mode(int mode, const T* x, const T* y, const int64_t* off, int64_t nseg,
                const int64_t* tbase, const int64_t* wtab, const uint32_t* status,
                const twofold_launch_t& lc, double* slots, void* out, hipStream_t st) {
#define TWOFOLD_SEG_MODE(A, MM) \
  return launch_seg<T, A, MM, DOT>(x, y, off, nseg, tbase, wtab, status, lc, slots, out, st)
  switch (mode) {
    case kPlain: TWOFOLD_SEG_MODE(T, kPlain);
    case kFast: TWOFOLD_SEG_MODE(T, kFast);
    case kRigorous: TWOFOLD_SEG_MODE(T, kRigorous);
    case kKahan: TWOFOLD_SEG_MODE(T, kKahan);
    case kFastRounded:
      if constexpr (DOT) TWOFOLD_SEG_MODE(T, kFastRounded);
      return TWOFOLD_EINVAL;
    case kRigorousRounded:
      if constexpr (DOT) TWOFOLD_SEG_MODE(T, kRigorousRounded);
      return TWOFOLD_EINVAL;
    case kWide:
      if constexpr (sizeof(T) == 4)
        TWOFOLD_SEG_MODE(double, kWide);
      else
        TWOFOLD_SEG_MODE(double, kDoubleDouble);
    case kMixed:
      if constexpr (sizeof(T) == 4) TWOFOLD_SEG_MODE(double, kMixed);
      return TWOFOLD_EINVAL;
    default: return TWOFOLD_EINVAL;
  }
#undef TWOFOLD_SEG_MODE
}

template <typename T, bool DOT>
int seg_entry(const T* x, const T* y, int64_t n_total, const int64_t* off, int64_t nseg, int mode,
              const twofold_launch_t* launch, void* out, void* ws, size_t ws_bytes, void* stream) {
  const int dtype = int(sizeof(T));
  if ((!x && n_total > 0) || !out || !off || (DOT && !y && n_total > 0) || !valid_count(n_total) ||
      !valid_count(nseg))
    return TWOFOLD_EINVAL;
  if (!mode_ok(dtype, DOT, mode)) return TWOFOLD_EINVAL;
  if (!elem_aligned(x, dtype) || (DOT && !elem_aligned(y, dtype)) ||
      !elem_aligned(out, out_f64(dtype, mode) ? 8 : 4) || !elem_aligned(off, 8))
    return TWOFOLD_EALIGN;
  twofold_launch_t lc;
  const int rc = resolve_seg(dtype, DOT, mode, n_total, nseg, launch, &lc);
  if (rc) return rc;
  if (nseg == 0) return TWOFOLD_OK;
  const int64_t nw = int64_t(lc.grid_blocks) * (lc.block_threads / 64);
  const SegLayout L = seg_layout(nseg, seg_max_tiles(n_total, nseg, lc.tile_elems), nw);
  if (!ws_ok(ws, ws_bytes, L.total)) return TWOFOLD_EWORKSPACE;
  char* base = static_cast<char*>(ws);
  uint32_t* status = reinterpret_cast<uint32_t*>(base);
  int64_t* tbase = reinterpret_cast<int64_t*>(base + L.tbase_off);
  double* slots = reinterpret_cast<double*>(base + L.slots_off);
  int64_t* rows = reinterpret_cast<int64_t*>(base + L.rows_off);
  uint32_t* bad = reinterpret_cast<uint32_t*>(base + L.bad_off);
  int64_t* wtab = nw <= kMaxSeqWaves ? reinterpret_cast<int64_t*>(base + L.wtab_off) : nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nrow = seg_rows(nseg);
  const dim3 grid(static_cast<unsigned>(nrow < kSegRowGrid ? nrow : kSegRowGrid));
  const dim3 block(static_cast<unsigned>(kSegRow));
  int rc2 = launch_kernel(seg_count_kernel, grid, block, st, off, nseg, n_total, lc.tile_elems,
                          tbase, rows, bad);
  if (!rc2) rc2 = launch_kernel(seg_rows_kernel, dim3(1), block, st, nrow, rows, bad, status);
  if (!rc2)
    rc2 = launch_kernel(seg_finish_kernel, grid, block, st, off, nseg, lc.tile_elems,
                        seg_tile_cost(dtype, DOT), tbase, rows, status, nw, wtab);
  if (rc2) return rc2;
  return seg_by_mode<T, DOT>(mode, x, y, off, nseg, tbase, wtab, status, lc, slots, out, st);
}

// Plans with at most this many waves carry a wave table (16 bytes a wave).
constexpr int64_t kMaxPlanWaves = int64_t(1) << 20;

// The wave table of a plan, from host offsets and tile table: for w = 0..NW,
// wt[2w] = the first tile whose start cost is at least floor(w*C/NW) and
// wt[2w+1] = the segment holding that tile (the last segment when the tile
// index is NT). Same cost model as the kernel's own search: a tile costs its
// length plus c0 = seg_tile_cost elements.
void build_wave_table(const int64_t* off, const int64_t* tb, int64_t nseg, int64_t ts, int64_t c0,
                      int64_t nw, int64_t* wt) {
  const int64_t C = (off[nseg] - off[0]) + c0 * tb[nseg];
  auto cbase = [&](int64_t s) { return (off[s] - off[0]) + c0 * tb[s]; };
  int64_t a = 0, sg = 0;
  for (int64_t w = 0; w <= nw; w++) {
    const int64_t lo = static_cast<int64_t>((static_cast<__int128>(w) * C) / nw);
    while (a + 1 < nseg && cbase(a + 1) <= lo) a++;
    const int64_t i = ((lo - cbase(a)) + ts + c0 - 1) / (ts + c0);
    const int64_t t = (i < tb[a + 1] - tb[a]) ? tb[a] + i : tb[a + 1];
    if (sg < a) sg = a;
    while (sg + 1 < nseg && tb[sg + 1] <= t) sg++;
    wt[2 * w] = t;
    wt[2 * w + 1] = sg;
  }
}

// Stream capture, as far as a call that is given no stream can see it. The
// legacy default stream reports a capture under way on any blocking
// stream (hipErrorStreamCaptureImplicit); a global-mode capture on a
// non-blocking stream shows up only as the allocator's refusal, one of the
// capture errors 900-908 of hip_runtime_api.h.
//
// The query and a refused allocation leave their error in the thread's HIP
// error state, where a later, unrelated launch check (torch's, say) would
// find it. Both are therefore cleared again, unless an error was already
// pending before plan creation made any HIP call (that one stays).
bool capture_under_way(bool state_was_clean) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(nullptr, &cs);
  if (e != hipSuccess && state_was_clean) (void)hipGetLastError();
  return e == hipErrorStreamCaptureImplicit ||
         (e == hipSuccess && cs != hipStreamCaptureStatusNone);
}

int refuse_capture(bool state_was_clean) {
  if (state_was_clean) (void)hipGetLastError();
  return TWOFOLD_ECAPTURE;
}

bool is_capture_error(hipError_t e) {
  return e >= hipErrorStreamCaptureUnsupported && e <= hipErrorStreamCaptureWrongThread;
}

}  // namespace

// A plan owns the device copies of the offsets, of the tile table and of
// the wave table; the caller's workspace holds the tile pairs.
struct twofold_seg_plan {
  int dtype, is_dot, mode;
  int64_t nseg, ntiles, n_total;
  twofold_launch_t lc;
  int64_t* d_off;
  int64_t* d_tbase;
  int64_t* d_wtab;  // null above kMaxPlanWaves waves: the kernel searches
};

extern "C" {

size_t twofold_workspace_bytes_seg(int dtype, int is_dot, int mode, int64_t n_total, int64_t nseg,
                                   const twofold_launch_t* launch) {
  if (!valid_dtype(dtype) || !valid_count(n_total) || !valid_count(nseg) ||
      !mode_ok(dtype, is_dot != 0, mode))
    return 0;
  twofold_launch_t lc;
  if (resolve_seg(dtype, is_dot != 0, mode, n_total, nseg, launch, &lc)) return 0;
  return seg_layout(nseg, seg_max_tiles(n_total, nseg, lc.tile_elems),
                    int64_t(lc.grid_blocks) * (lc.block_threads / 64))
      .total;
}

int twofold_segsum_f32(const float* x, int64_t n_total, const int64_t* offsets, int64_t nseg,
                       int mode, const twofold_launch_t* launch, twofold_f32_t* out, void* ws,
                       size_t ws_bytes, void* stream) {
  // binary64 results: twofold_segsumd_f32, twofold_segsum_mixed_f32
  if (mode == kWide || mode == kMixed) return TWOFOLD_EINVAL;
  return seg_entry<float, false>(x, nullptr, n_total, offsets, nseg, mode, launch, out, ws, ws_bytes,
                                 stream);
}
int twofold_segsum_f64(const double* x, int64_t n_total, const int64_t* offsets, int64_t nseg,
                       int mode, const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                       size_t ws_bytes, void* stream) {
  return seg_entry<double, false>(x, nullptr, n_total, offsets, nseg, mode, launch, out, ws, ws_bytes,
                                  stream);
}
int twofold_segdot_f32(const float* x, const float* y, int64_t n_total, const int64_t* offsets,
                       int64_t nseg, int mode, const twofold_launch_t* launch, twofold_f32_t* out,
                       void* ws, size_t ws_bytes, void* stream) {
  // binary64 results: twofold_segdotd_f32, twofold_segdot_mixed_f32
  if (mode == kWide || mode == kMixed) return TWOFOLD_EINVAL;
  return seg_entry<float, true>(x, y, n_total, offsets, nseg, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_segdot_f64(const double* x, const double* y, int64_t n_total, const int64_t* offsets,
                       int64_t nseg, int mode, const twofold_launch_t* launch, twofold_f64_t* out,
                       void* ws, size_t ws_bytes, void* stream) {
  return seg_entry<double, true>(x, y, n_total, offsets, nseg, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_segsumd_f32(const float* x, int64_t n_total, const int64_t* offsets, int64_t nseg,
                        const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                        size_t ws_bytes, void* stream) {
  return seg_entry<float, false>(x, nullptr, n_total, offsets, nseg, kWide, launch, out, ws,
                                 ws_bytes, stream);
}
int twofold_segsumd_f64(const double* x, int64_t n_total, const int64_t* offsets, int64_t nseg,
                        const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                        size_t ws_bytes, void* stream) {
  return seg_entry<double, false>(x, nullptr, n_total, offsets, nseg, kWide, launch, out, ws,
                                  ws_bytes, stream);
}
int twofold_segdotd_f32(const float* x, const float* y, int64_t n_total, const int64_t* offsets,
                        int64_t nseg, const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                        size_t ws_bytes, void* stream) {
  return seg_entry<float, true>(x, y, n_total, offsets, nseg, kWide, launch, out, ws, ws_bytes,
                                stream);
}
int twofold_segdotd_f64(const double* x, const double* y, int64_t n_total, const int64_t* offsets,
                        int64_t nseg, const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                        size_t ws_bytes, void* stream) {
  return seg_entry<double, true>(x, y, n_total, offsets, nseg, kWide, launch, out, ws, ws_bytes,
                                 stream);
}
int twofold_segsum_mixed_f32(const float* x, int64_t n_total, const int64_t* offsets,
                             int64_t nseg, const twofold_launch_t* launch, twofold_f64_t* out,
                             void* ws, size_t ws_bytes, void* stream) {
  return seg_entry<float, false>(x, nullptr, n_total, offsets, nseg, kMixed, launch, out, ws,
                                 ws_bytes, stream);
}
int twofold_segdot_mixed_f32(const float* x, const float* y, int64_t n_total,
                             const int64_t* offsets, int64_t nseg, const twofold_launch_t* launch,
                             twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream) {
  return seg_entry<float, true>(x, y, n_total, offsets, nseg, kMixed, launch, out, ws, ws_bytes,
                                stream);
}

int twofold_seg_plan_create(const int64_t* offsets_host, int64_t nseg, int dtype, int is_dot,
                            int mode, const twofold_launch_t* launch, twofold_seg_plan_t** plan) {
  if (!plan) return TWOFOLD_EINVAL;
  *plan = nullptr;
  if (!offsets_host || !valid_count(nseg) || !valid_dtype(dtype)) return TWOFOLD_EINVAL;
  if (!mode_ok(dtype, is_dot != 0, mode)) return TWOFOLD_EINVAL;
  if (offsets_host[0] != 0) return TWOFOLD_EOFFSETS;
  for (int64_t s = 0; s < nseg; s++)
    if (offsets_host[s + 1] < offsets_host[s]) return TWOFOLD_EOFFSETS;
  const int64_t n_total = offsets_host[nseg];
  if (!valid_count(n_total)) return TWOFOLD_EINVAL;
  twofold_launch_t lc;
  const int rc = resolve_seg(dtype, is_dot != 0, mode, n_total, nseg, launch, &lc);
  if (rc) return rc;
  int64_t* tb = static_cast<int64_t*>(malloc(sizeof(int64_t) * size_t(nseg + 1)));
  if (!tb) return TWOFOLD_EINVAL;
  int64_t acc = 0;
  for (int64_t s = 0; s < nseg; s++) {
    tb[s] = acc;
    const int64_t len = offsets_host[s + 1] - offsets_host[s];
    acc += (len + lc.tile_elems - 1) / lc.tile_elems;
  }
  tb[nseg] = acc;
  const bool state_was_clean = hipPeekAtLastError() == hipSuccess;
  if (capture_under_way(state_was_clean)) {
    free(tb);
    return refuse_capture(state_was_clean);
  }
  twofold_seg_plan* p = static_cast<twofold_seg_plan*>(calloc(1, sizeof(twofold_seg_plan)));
  if (!p) {
    free(tb);
    return TWOFOLD_EINVAL;
  }
  p->dtype = dtype;
  p->is_dot = is_dot != 0;
  p->mode = mode;
  p->nseg = nseg;
  p->ntiles = acc;
  p->n_total = n_total;
  p->lc = lc;
  const size_t bytes = sizeof(int64_t) * size_t(nseg + 1);
  const int64_t nw = int64_t(lc.grid_blocks) * (lc.block_threads / 64);
  int64_t* wt = nullptr;
  size_t wbytes = 0;
  bool ok = true;
  if (nseg > 0 && nw <= kMaxPlanWaves) {
    wbytes = sizeof(int64_t) * size_t(2 * (nw + 1));
    wt = static_cast<int64_t*>(malloc(wbytes));
    ok = wt != nullptr;
    if (ok)
      build_wave_table(offsets_host, tb, nseg, lc.tile_elems, seg_tile_cost(dtype, is_dot != 0),
                       nw, wt);
  }
  // the first failing HIP call's error, if any
  hipError_t he = hipSuccess;
  auto run = [&](hipError_t e) {
    if (he == hipSuccess) he = e;
    return e == hipSuccess;
  };
  ok = ok && run(hipMalloc(reinterpret_cast<void**>(&p->d_off), bytes)) &&
       run(hipMalloc(reinterpret_cast<void**>(&p->d_tbase), bytes)) &&
       run(hipMemcpy(p->d_off, offsets_host, bytes, hipMemcpyHostToDevice)) &&
       run(hipMemcpy(p->d_tbase, tb, bytes, hipMemcpyHostToDevice));
  if (ok && wt)
    ok = run(hipMalloc(reinterpret_cast<void**>(&p->d_wtab), wbytes)) &&
         run(hipMemcpy(p->d_wtab, wt, wbytes, hipMemcpyHostToDevice));
  free(tb);
  free(wt);
  if (!ok) {
    if (p->d_off) (void)hipFree(p->d_off);
    if (p->d_tbase) (void)hipFree(p->d_tbase);
    if (p->d_wtab) (void)hipFree(p->d_wtab);
    free(p);
    if (he == hipSuccess) return TWOFOLD_EINVAL;  // host allocation failed
    return is_capture_error(he) ? refuse_capture(state_was_clean) : TWOFOLD_EHIP;
  }
  *plan = p;
  return TWOFOLD_OK;
}

size_t twofold_seg_plan_workspace_bytes(const twofold_seg_plan_t* plan) {
  if (!plan) return 0;
  return align256(size_t(16) * size_t(plan->ntiles > 0 ? plan->ntiles : 1));
}

int twofold_seg_plan_get_launch(const twofold_seg_plan_t* plan, twofold_launch_t* out) {
  if (!plan || !out) return TWOFOLD_EINVAL;
  *out = plan->lc;
  return TWOFOLD_OK;
}

int twofold_seg_plan_execute(const twofold_seg_plan_t* plan, const void* x, const void* y,
                             void* out, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !out) return TWOFOLD_EINVAL;
  if (plan->n_total > 0 && (!x || (plan->is_dot && !y))) return TWOFOLD_EINVAL;
  if (!plan->is_dot && y) return TWOFOLD_EINVAL;
  const int dtype = plan->dtype;
  if (!elem_aligned(x, dtype) || (y && !elem_aligned(y, dtype)) ||
      !elem_aligned(out, out_f64(dtype, plan->mode) ? 8 : 4))
    return TWOFOLD_EALIGN;
  if (plan->nseg == 0) return TWOFOLD_OK;
  if (!ws_ok(ws, ws_bytes, twofold_seg_plan_workspace_bytes(plan))) return TWOFOLD_EWORKSPACE;
  double* slots = static_cast<double*>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t* off = plan->d_off;
  const int64_t* tb = plan->d_tbase;
  const int64_t* wt = plan->d_wtab;
  const int64_t ns = plan->nseg;
  const twofold_launch_t& lc = plan->lc;
  if (dtype == 4) {
    const float* xf = static_cast<const float*>(x);
    const float* yf = static_cast<const float*>(y);
    if (plan->is_dot)
      return seg_by_mode<float, true>(plan->mode, xf, yf, off, ns, tb, wt, nullptr, lc, slots, out,
                                      st);
    return seg_by_mode<float, false>(plan->mode, xf, yf, off, ns, tb, wt, nullptr, lc, slots, out,
                                     st);
  }
  const double* xd = static_cast<const double*>(x);
  const double* yd = static_cast<const double*>(y);
  if (plan->is_dot)
    return seg_by_mode<double, true>(plan->mode, xd, yd, off, ns, tb, wt, nullptr, lc, slots, out,
                                     st);
  return seg_by_mode<double, false>(plan->mode, xd, yd, off, ns, tb, wt, nullptr, lc, slots, out,
                                    st);
}

int twofold_seg_plan_destroy(twofold_seg_plan_t* plan) {
  if (!plan) return TWOFOLD_OK;
  int rc = TWOFOLD_OK;
  if (plan->d_off && hipFree(plan->d_off) != hipSuccess) rc = TWOFOLD_EHIP;
  if (plan->d_tbase && hipFree(plan->d_tbase) != hipSuccess) rc = TWOFOLD_EHIP;
  if (plan->d_wtab && hipFree(plan->d_wtab) != hipSuccess) rc = TWOFOLD_EHIP;
  free(plan);
  return rc;
}

}  // extern "C"
