// twofold.hip: host side of the C interface declared in include/twofold.h.
//
// Argument checks run on the host before any HIP call; launches go to the
// caller's stream; nothing on the execute path allocates, frees or
// synchronises, so every execute call can be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "kernels.hpp"
#include "twofold.h"

using namespace twofold;

namespace {

constexpr size_t kHdrBytes = 256;
constexpr int64_t kMaxGrid = int64_t(1) << 20;
constexpr int64_t kMaxTile = int64_t(1) << 30;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

bool valid_dtype(int dtype) { return dtype == 4 || dtype == 8; }

// Tuned defaults. Generated table first (kind, dtype, is_dot, mode, n_max,
// block_threads, unroll, max_blocks, tile_elems), searched in order; the
// fallback below applies when no row matches.
struct TuneRow {
  int kind, dtype, is_dot, mode;
  int64_t n_max;
  int block_threads, unroll, max_blocks;
  int64_t tile_elems;
};
const TuneRow kTuned[] = {
#include "tuned_table.inc"
};

twofold_launch_t lookup(int kind, int dtype, int is_dot, int mode, int64_t n) {
  twofold_launch_t lc;
  memset(&lc, 0, sizeof lc);
  lc.block_threads = 256;
  lc.unroll = 4;
  lc.grid_blocks = kind == 0 ? 2048 : 1024;
  lc.tile_elems = (dtype == 4 ? 8192 : 4096);
  for (const TuneRow& r : kTuned) {
    if (r.kind == kind && r.dtype == dtype && r.is_dot == is_dot && r.mode == mode && n <= r.n_max) {
      lc.block_threads = r.block_threads;
      lc.unroll = r.unroll;
      lc.grid_blocks = r.max_blocks;
      lc.tile_elems = r.tile_elems;
      break;
    }
  }
  return lc;
}

bool valid_unroll(int u) { return u == 1 || u == 2 || u == 4 || u == 8; }

// Resolve a single-vector launch: zero fields take the tuned default; with
// no explicit grid the grid is the blocks needed for one round, capped at
// the tuned maximum.
int resolve_single(int dtype, int is_dot, int mode, int64_t n, const twofold_launch_t* in,
                   twofold_launch_t* lc) {
  twofold_launch_t d = lookup(0, dtype, is_dot, mode, n);
  twofold_launch_t r = d;
  if (in) {
    if (in->reserved != 0) return TWOFOLD_EINVAL;
    if (in->block_threads) r.block_threads = in->block_threads;
    if (in->unroll) r.unroll = in->unroll;
    r.grid_blocks = in->grid_blocks;
  } else {
    r.grid_blocks = 0;
  }
  if (r.block_threads < 64 || r.block_threads > 1024 || r.block_threads % 64) return TWOFOLD_EINVAL;
  if (!valid_unroll(r.unroll)) return TWOFOLD_EINVAL;
  if (r.grid_blocks == 0) {
    const int64_t W = 16 / dtype;
    const int64_t nv = (n + W - 1) / W;
    const int64_t per_block = int64_t(r.block_threads) * r.unroll;
    int64_t gb = (nv + per_block - 1) / per_block;
    if (gb > d.grid_blocks) gb = d.grid_blocks;
    if (gb < 1) gb = 1;
    r.grid_blocks = static_cast<int32_t>(gb);
  }
  if (r.grid_blocks < 1 || r.grid_blocks > kMaxGrid) return TWOFOLD_EINVAL;
  r.tile_elems = 0;
  *lc = r;
  return TWOFOLD_OK;
}

int resolve_seg(int dtype, int is_dot, int mode, int64_t n_total, const twofold_launch_t* in,
                twofold_launch_t* lc) {
  twofold_launch_t r = lookup(1, dtype, is_dot, mode, n_total);
  if (in) {
    if (in->reserved != 0) return TWOFOLD_EINVAL;
    if (in->block_threads) r.block_threads = in->block_threads;
    if (in->unroll) r.unroll = in->unroll;
    if (in->grid_blocks) r.grid_blocks = in->grid_blocks;
    if (in->tile_elems) r.tile_elems = in->tile_elems;
  }
  if (r.block_threads < 64 || r.block_threads > 1024 || r.block_threads % 64) return TWOFOLD_EINVAL;
  if (!valid_unroll(r.unroll)) return TWOFOLD_EINVAL;
  if (r.grid_blocks < 1 || r.grid_blocks > kMaxGrid) return TWOFOLD_EINVAL;
  const int64_t quantum = 64 * (16 / dtype);
  if (r.tile_elems <= 0 || r.tile_elems > kMaxTile || r.tile_elems % quantum) return TWOFOLD_EINVAL;
  *lc = r;
  return TWOFOLD_OK;
}

// Single vector: the GB block pairs (binary64) when GB > 1.
size_t single_ws_bytes(const twofold_launch_t& lc) {
  return align256(size_t(16) * size_t(lc.grid_blocks));
}

struct SegLayout {
  size_t tbase_off, slots_off, total;
};

// Device-offset path: [status word][tile table][tile pairs]; the tiling
// kernel rewrites the status and the table on every call.
SegLayout seg_layout(int64_t nseg, int64_t max_tiles) {
  SegLayout L;
  L.tbase_off = kHdrBytes;
  L.slots_off = L.tbase_off + align256(size_t(8) * size_t(nseg + 1));
  L.total = L.slots_off + align256(size_t(16) * size_t(max_tiles));
  return L;
}

int64_t seg_max_tiles(int64_t n_total, int64_t nseg, int64_t ts) {
  return (n_total + ts - 1) / ts + nseg;
}

bool elem_aligned(const void* p, int dtype) {
  return (reinterpret_cast<uintptr_t>(p) % uintptr_t(dtype)) == 0;
}

int launch_status() {
  const hipError_t err = hipGetLastError();
  return err == hipSuccess ? TWOFOLD_OK : TWOFOLD_EHIP;
}

// ---- kernel dispatch ---------------------------------------------------------

template <typename T, typename A, int M, bool DOT, bool YV>
int launch_single_u(const T* x, const T* y, int64_t n, const twofold_launch_t& lc, double* part,
                    void* out, hipStream_t st) {
  const dim3 grid(lc.grid_blocks), block(lc.block_threads);
  switch (lc.unroll) {
    case 1: single_kernel<T, A, M, DOT, YV, 1><<<grid, block, 0, st>>>(x, y, n, part, out); break;
    case 2: single_kernel<T, A, M, DOT, YV, 2><<<grid, block, 0, st>>>(x, y, n, part, out); break;
    case 4: single_kernel<T, A, M, DOT, YV, 4><<<grid, block, 0, st>>>(x, y, n, part, out); break;
    default: single_kernel<T, A, M, DOT, YV, 8><<<grid, block, 0, st>>>(x, y, n, part, out); break;
  }
  if (launch_status()) return TWOFOLD_EHIP;
  if (lc.grid_blocks > 1) {
    single_pass2_kernel<T, M><<<dim3(1), dim3(kPass2Lanes), 0, st>>>(part, lc.grid_blocks, out);
    return launch_status();
  }
  return TWOFOLD_OK;
}

template <typename T, typename A, int M, bool DOT>
int launch_single(const T* x, const T* y, int64_t n, const twofold_launch_t& lc, double* part,
                  void* out, hipStream_t st) {
  if constexpr (DOT) {
    const bool yv = ((reinterpret_cast<uintptr_t>(y) - reinterpret_cast<uintptr_t>(x)) & 15u) == 0;
    if (!yv) return launch_single_u<T, A, M, DOT, false>(x, y, n, lc, part, out, st);
  }
  return launch_single_u<T, A, M, DOT, true>(x, y, n, lc, part, out, st);
}

template <typename T, typename A, int M, bool DOT, bool YV>
int launch_seg_u(const T* x, const T* y, const int64_t* off, int64_t nseg, const int64_t* tbase,
                 const uint32_t* status, const twofold_launch_t& lc, double* slots, void* out,
                 hipStream_t st) {
  const dim3 grid(lc.grid_blocks), block(lc.block_threads);
  const int64_t ts = lc.tile_elems;
#define TWOFOLD_SEG(UU)                                                                       \
  seg_kernel<T, A, M, DOT, YV, UU><<<grid, block, 0, st>>>(x, y, off, nseg, tbase, ts, status, \
                                                           slots, out)
  switch (lc.unroll) {
    case 1: TWOFOLD_SEG(1); break;
    case 2: TWOFOLD_SEG(2); break;
    case 4: TWOFOLD_SEG(4); break;
    default: TWOFOLD_SEG(8); break;
  }
#undef TWOFOLD_SEG
  if (launch_status()) return TWOFOLD_EHIP;
  const int64_t blocks2 = (nseg + 3) / 4;  // one wave per segment, 4 waves per block
  seg_pass2_kernel<T, M><<<dim3(unsigned(blocks2)), dim3(256), 0, st>>>(tbase, nseg, status, slots,
                                                                        out);
  return launch_status();
}

template <typename T, typename A, int M, bool DOT>
int launch_seg(const T* x, const T* y, const int64_t* off, int64_t nseg, const int64_t* tbase,
               const uint32_t* status, const twofold_launch_t& lc, double* slots, void* out,
               hipStream_t st) {
  if constexpr (DOT) {
    const bool yv = ((reinterpret_cast<uintptr_t>(y) - reinterpret_cast<uintptr_t>(x)) & 15u) == 0;
    if (!yv)
      return launch_seg_u<T, A, M, DOT, false>(x, y, off, nseg, tbase, status, lc, slots, out, st);
  }
  return launch_seg_u<T, A, M, DOT, true>(x, y, off, nseg, tbase, status, lc, slots, out, st);
}

// Mode switch for one data type. WIDE is only meaningful for binary32 data.
template <typename T, bool DOT>
int single_by_mode(int mode, const T* x, const T* y, int64_t n, const twofold_launch_t& lc,
                   double* part, void* out, hipStream_t st) {
  switch (mode) {
    case kPlain: return launch_single<T, T, kPlain, DOT>(x, y, n, lc, part, out, st);
    case kFast: return launch_single<T, T, kFast, DOT>(x, y, n, lc, part, out, st);
    case kRigorous: return launch_single<T, T, kRigorous, DOT>(x, y, n, lc, part, out, st);
    default:
      if constexpr (sizeof(T) == 4)
        return launch_single<T, double, kWide, DOT>(x, y, n, lc, part, out, st);
      return TWOFOLD_EINVAL;
  }
}

template <typename T, bool DOT>
int seg_by_mode(int mode, const T* x, const T* y, const int64_t* off, int64_t nseg,
                const int64_t* tbase, const uint32_t* status, const twofold_launch_t& lc,
                double* slots, void* out, hipStream_t st) {
  switch (mode) {
    case kPlain:
      return launch_seg<T, T, kPlain, DOT>(x, y, off, nseg, tbase, status, lc, slots, out, st);
    case kFast:
      return launch_seg<T, T, kFast, DOT>(x, y, off, nseg, tbase, status, lc, slots, out, st);
    case kRigorous:
      return launch_seg<T, T, kRigorous, DOT>(x, y, off, nseg, tbase, status, lc, slots, out, st);
    default:
      if constexpr (sizeof(T) == 4)
        return launch_seg<T, double, kWide, DOT>(x, y, off, nseg, tbase, status, lc, slots, out, st);
      return TWOFOLD_EINVAL;
  }
}

// Common body of the single-vector entry points.
template <typename T, bool DOT>
int single_entry(const T* x, const T* y, int64_t n, int mode, const twofold_launch_t* launch,
                 void* out, void* ws, size_t ws_bytes, void* stream) {
  const int dtype = int(sizeof(T));
  // Data pointers may be NULL only when there is no data (torch hands out
  // NULL for empty tensors).
  if ((!x && n > 0) || !out || (DOT && !y && n > 0) || n < 0) return TWOFOLD_EINVAL;
  if (mode < kPlain || mode > kWide || (mode == kWide && dtype != 4)) return TWOFOLD_EINVAL;
  if (!elem_aligned(x, dtype) || (DOT && !elem_aligned(y, dtype))) return TWOFOLD_EALIGN;
  if (!elem_aligned(out, mode == kWide ? 8 : dtype)) return TWOFOLD_EALIGN;
  twofold_launch_t lc;
  const int rc = resolve_single(dtype, DOT, mode, n, launch, &lc);
  if (rc) return rc;
  if (lc.grid_blocks > 1 &&
      (!ws || ws_bytes < single_ws_bytes(lc) || (reinterpret_cast<uintptr_t>(ws) & 255u)))
    return TWOFOLD_EWORKSPACE;
  return single_by_mode<T, DOT>(mode, x, y, n, lc, static_cast<double*>(ws), out,
                                static_cast<hipStream_t>(stream));
}

template <typename T, bool DOT>
int seg_entry(const T* x, const T* y, int64_t n_total, const int64_t* off, int64_t nseg, int mode,
              const twofold_launch_t* launch, void* out, void* ws, size_t ws_bytes, void* stream) {
  const int dtype = int(sizeof(T));
  if ((!x && n_total > 0) || !out || !off || (DOT && !y && n_total > 0) || n_total < 0 || nseg < 0)
    return TWOFOLD_EINVAL;
  if (mode < kPlain || mode > kRigorous) return TWOFOLD_EINVAL;
  if (!elem_aligned(x, dtype) || (DOT && !elem_aligned(y, dtype)) || !elem_aligned(out, dtype) ||
      !elem_aligned(off, 8))
    return TWOFOLD_EALIGN;
  twofold_launch_t lc;
  const int rc = resolve_seg(dtype, DOT, mode, n_total, launch, &lc);
  if (rc) return rc;
  if (nseg == 0) return TWOFOLD_OK;
  const SegLayout L = seg_layout(nseg, seg_max_tiles(n_total, nseg, lc.tile_elems));
  if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255u)) return TWOFOLD_EWORKSPACE;
  char* base = static_cast<char*>(ws);
  uint32_t* status = reinterpret_cast<uint32_t*>(base);
  int64_t* tbase = reinterpret_cast<int64_t*>(base + L.tbase_off);
  double* slots = reinterpret_cast<double*>(base + L.slots_off);
  hipStream_t st = static_cast<hipStream_t>(stream);
  seg_tiles_kernel<<<1, 1024, 0, st>>>(off, nseg, n_total, lc.tile_elems, tbase, status);
  if (launch_status()) return TWOFOLD_EHIP;
  return seg_by_mode<T, DOT>(mode, x, y, off, nseg, tbase, status, lc, slots, out, st);
}

}  // namespace

// ---- plans -------------------------------------------------------------------

// A plan owns the device copies of the offsets and of the tile table; the
// caller's workspace holds the tile pairs.
struct twofold_seg_plan {
  int dtype, is_dot, mode;
  int64_t nseg, ntiles, n_total;
  twofold_launch_t lc;
  int64_t* d_off;
  int64_t* d_tbase;
};

extern "C" {

int twofold_default_launch(int kind, int dtype, int is_dot, int mode, int64_t n, int64_t nseg,
                           twofold_launch_t* out) {
  if (!out || !valid_dtype(dtype) || (kind != 0 && kind != 1) || n < 0 || nseg < 0)
    return TWOFOLD_EINVAL;
  if (mode < kPlain || mode > kWide || (mode == kWide && dtype != 4)) return TWOFOLD_EINVAL;
  if (kind == 0) return resolve_single(dtype, is_dot != 0, mode, n, nullptr, out);
  return resolve_seg(dtype, is_dot != 0, mode, n, nullptr, out);
}

size_t twofold_workspace_bytes_single(int dtype, int is_dot, int mode, int64_t n,
                                      const twofold_launch_t* launch) {
  if (!valid_dtype(dtype) || n < 0) return 0;
  twofold_launch_t lc;
  if (resolve_single(dtype, is_dot != 0, mode, n, launch, &lc)) return 0;
  return single_ws_bytes(lc);
}

size_t twofold_workspace_bytes_seg(int dtype, int is_dot, int mode, int64_t n_total, int64_t nseg,
                                   const twofold_launch_t* launch) {
  if (!valid_dtype(dtype) || n_total < 0 || nseg < 0) return 0;
  twofold_launch_t lc;
  if (resolve_seg(dtype, is_dot != 0, mode, n_total, launch, &lc)) return 0;
  return seg_layout(nseg, seg_max_tiles(n_total, nseg, lc.tile_elems)).total;
}

int twofold_sum_f32(const float* x, int64_t n, int mode, const twofold_launch_t* launch,
                    twofold_f32_t* out, void* ws, size_t ws_bytes, void* stream) {
  if (mode == kWide) return TWOFOLD_EINVAL;
  return single_entry<float, false>(x, nullptr, n, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_sum_f64(const double* x, int64_t n, int mode, const twofold_launch_t* launch,
                    twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream) {
  return single_entry<double, false>(x, nullptr, n, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_dot_f32(const float* x, const float* y, int64_t n, int mode,
                    const twofold_launch_t* launch, twofold_f32_t* out, void* ws, size_t ws_bytes,
                    void* stream) {
  if (mode == kWide) return TWOFOLD_EINVAL;
  return single_entry<float, true>(x, y, n, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_dot_f64(const double* x, const double* y, int64_t n, int mode,
                    const twofold_launch_t* launch, twofold_f64_t* out, void* ws, size_t ws_bytes,
                    void* stream) {
  return single_entry<double, true>(x, y, n, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_sumd_f32(const float* x, int64_t n, const twofold_launch_t* launch, twofold_f64_t* out,
                     void* ws, size_t ws_bytes, void* stream) {
  return single_entry<float, false>(x, nullptr, n, kWide, launch, out, ws, ws_bytes, stream);
}
int twofold_dotd_f32(const float* x, const float* y, int64_t n, const twofold_launch_t* launch,
                     twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream) {
  return single_entry<float, true>(x, y, n, kWide, launch, out, ws, ws_bytes, stream);
}

int twofold_segsum_f32(const float* x, int64_t n_total, const int64_t* offsets, int64_t nseg,
                       int mode, const twofold_launch_t* launch, twofold_f32_t* out, void* ws,
                       size_t ws_bytes, void* stream) {
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
  return seg_entry<float, true>(x, y, n_total, offsets, nseg, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_segdot_f64(const double* x, const double* y, int64_t n_total, const int64_t* offsets,
                       int64_t nseg, int mode, const twofold_launch_t* launch, twofold_f64_t* out,
                       void* ws, size_t ws_bytes, void* stream) {
  return seg_entry<double, true>(x, y, n_total, offsets, nseg, mode, launch, out, ws, ws_bytes, stream);
}

int twofold_seg_plan_create(const int64_t* offsets_host, int64_t nseg, int dtype, int is_dot,
                            int mode, const twofold_launch_t* launch, twofold_seg_plan_t** plan) {
  if (!plan) return TWOFOLD_EINVAL;
  *plan = nullptr;
  if (!offsets_host || nseg < 0 || !valid_dtype(dtype)) return TWOFOLD_EINVAL;
  if (mode < kPlain || mode > kWide || (mode == kWide && dtype != 4)) return TWOFOLD_EINVAL;
  if (offsets_host[0] != 0) return TWOFOLD_EOFFSETS;
  for (int64_t s = 0; s < nseg; s++)
    if (offsets_host[s + 1] < offsets_host[s]) return TWOFOLD_EOFFSETS;
  const int64_t n_total = offsets_host[nseg];
  twofold_launch_t lc;
  const int rc = resolve_seg(dtype, is_dot != 0, mode, n_total, launch, &lc);
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
  bool ok = hipMalloc(reinterpret_cast<void**>(&p->d_off), bytes) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&p->d_tbase), bytes) == hipSuccess &&
            hipMemcpy(p->d_off, offsets_host, bytes, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(p->d_tbase, tb, bytes, hipMemcpyHostToDevice) == hipSuccess;
  free(tb);
  if (!ok) {
    if (p->d_off) (void)hipFree(p->d_off);
    if (p->d_tbase) (void)hipFree(p->d_tbase);
    free(p);
    return TWOFOLD_EHIP;
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
  const bool f64out = dtype == 8 || plan->mode == kWide;
  if (!elem_aligned(x, dtype) || (y && !elem_aligned(y, dtype)) || !elem_aligned(out, f64out ? 8 : 4))
    return TWOFOLD_EALIGN;
  if (plan->nseg == 0) return TWOFOLD_OK;
  if (!ws || ws_bytes < twofold_seg_plan_workspace_bytes(plan) ||
      (reinterpret_cast<uintptr_t>(ws) & 255u))
    return TWOFOLD_EWORKSPACE;
  double* slots = static_cast<double*>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t* off = plan->d_off;
  const int64_t* tb = plan->d_tbase;
  const int64_t ns = plan->nseg;
  const twofold_launch_t& lc = plan->lc;
  if (dtype == 4) {
    const float* xf = static_cast<const float*>(x);
    const float* yf = static_cast<const float*>(y);
    if (plan->is_dot)
      return seg_by_mode<float, true>(plan->mode, xf, yf, off, ns, tb, nullptr, lc, slots, out, st);
    return seg_by_mode<float, false>(plan->mode, xf, yf, off, ns, tb, nullptr, lc, slots, out, st);
  }
  const double* xd = static_cast<const double*>(x);
  const double* yd = static_cast<const double*>(y);
  if (plan->is_dot)
    return seg_by_mode<double, true>(plan->mode, xd, yd, off, ns, tb, nullptr, lc, slots, out, st);
  return seg_by_mode<double, false>(plan->mode, xd, yd, off, ns, tb, nullptr, lc, slots, out, st);
}

int twofold_seg_plan_destroy(twofold_seg_plan_t* plan) {
  if (!plan) return TWOFOLD_OK;
  int rc = TWOFOLD_OK;
  if (plan->d_off && hipFree(plan->d_off) != hipSuccess) rc = TWOFOLD_EHIP;
  if (plan->d_tbase && hipFree(plan->d_tbase) != hipSuccess) rc = TWOFOLD_EHIP;
  free(plan);
  return rc;
}

const char* twofold_strerror(int status) {
  switch (status) {
    case TWOFOLD_OK: return "ok";
    case TWOFOLD_EINVAL: return "invalid argument";
    case TWOFOLD_EWORKSPACE: return "workspace missing, misaligned or too small";
    case TWOFOLD_EHIP: return "HIP runtime error";
    case TWOFOLD_EALIGN: return "data pointer not aligned to its element size";
    case TWOFOLD_EOFFSETS: return "segment offsets must start at 0 and not decrease";
    default: return "unknown status";
  }
}

}  // extern "C"
