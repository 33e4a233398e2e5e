// batch.hip: a mixed batch of sums and dots in one launch (twofold_batch in
// include/twofold.h). Items may differ in data type, operation and form
// (every form, the binary64-result ones included);
// each is reduced exactly as its single-vector call with the batch's launch
// (steps 1-8), so its pair is that call's, bit for bit. The per-item form is
// a uniform branch at the item's start: every block takes the same path.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>

#include "host_common.hpp"
#include "kernels.hpp"
#include "twofold.h"

namespace twofold {

constexpr int kMaxBatch = 64;

// One item as the kernels see it. kind = f64 | dot << 1 | yv << 2 | mode << 3.
struct BatchEntry {
  const void* x;
  const void* y;
  void* out;
  int64_t n;
  int64_t kind;
};

struct BatchArgs {
  BatchEntry e[kMaxBatch];
};

template <typename T, bool DOT, bool YV, int U, int BMAX>
__device__ __forceinline__ void batch_item(const BatchEntry& b, int mode, double* part) {
  const T* x = static_cast<const T*>(b.x);
  const T* y = static_cast<const T*>(b.y);
  constexpr bool AH = rounds_ahead<BMAX, DOT, U>();
  switch (mode) {
    case kPlain: single_block<T, T, kPlain, DOT, YV, U, AH>(x, y, b.n, part, b.out, 0); break;
    case kFast: single_block<T, T, kFast, DOT, YV, U, AH>(x, y, b.n, part, b.out, 0); break;
    case kRigorous: single_block<T, T, kRigorous, DOT, YV, U, AH>(x, y, b.n, part, b.out, 0); break;
    case kKahan: single_block<T, T, kKahan, DOT, YV, U, AH>(x, y, b.n, part, b.out, 0); break;
    case kFastRounded:
      if constexpr (DOT) single_block<T, T, kFastRounded, DOT, YV, U, AH>(x, y, b.n, part, b.out, 0);
      break;
    default:
      if constexpr (DOT) single_block<T, T, kRigorousRounded, DOT, YV, U, AH>(x, y, b.n, part, b.out, 0);
      break;
  }
}

template <typename T, int U, int BMAX>
__device__ __forceinline__ void batch_by_op(const BatchEntry& b, int64_t kind, double* part) {
  const int mode = static_cast<int>(kind >> 3);
  if (kind & 2) {
    if (kind & 4)
      batch_item<T, true, true, U, BMAX>(b, mode, part);
    else
      batch_item<T, true, false, U, BMAX>(b, mode, part);
  } else {
    batch_item<T, false, true, U, BMAX>(b, mode, part);
  }
}

// Pass 1: sets of gridDim.x blocks as in the multi-vector kernel; item v's
// block pairs at part[v * gridDim.x ...].
template <int U, int BMAX>
__global__ void __launch_bounds__(BMAX)
batch_kernel(const BatchArgs args, int count, double* __restrict__ part) {
  for (int v = blockIdx.y; v < count; v += gridDim.y) {
    const BatchEntry& b = args.e[v];
    double* p = part + 2 * static_cast<int64_t>(v) * gridDim.x;
    if (b.kind & 1)
      batch_by_op<double, U, BMAX>(b, b.kind, p);
    else
      batch_by_op<float, U, BMAX>(b, b.kind, p);
    __syncthreads();  // the block combine's LDS is reused for the next item
  }
}

// Items with binary64 results: the wider accumulator (binary64 for binary32
// data, double-word for binary64 data) and the mixed form (binary32 data).
// A kernel of their own, so that batches of same-type forms keep the leaner
// kernel above.
template <bool DOT, bool YV, int U, int BMAX>
__device__ __forceinline__ void batch_item_wide(const BatchEntry& b, int64_t kind, double* part) {
  constexpr bool AH = rounds_ahead<BMAX, DOT, U>();
  if (kind & 1) {
    single_block<double, double, kDoubleDouble, DOT, YV, U, AH>(
        static_cast<const double*>(b.x), static_cast<const double*>(b.y), b.n, part, b.out, 0);
  } else if ((kind >> 3) == kMixed) {
    single_block<float, double, kMixed, DOT, YV, U, AH>(
        static_cast<const float*>(b.x), static_cast<const float*>(b.y), b.n, part, b.out, 0);
  } else {
    single_block<float, double, kWide, DOT, YV, U, AH>(
        static_cast<const float*>(b.x), static_cast<const float*>(b.y), b.n, part, b.out, 0);
  }
}

template <int U, int BMAX>
__global__ void __launch_bounds__(BMAX)
batch_kernel_wide(const BatchArgs args, int count, double* __restrict__ part) {
  for (int v = blockIdx.y; v < count; v += gridDim.y) {
    const BatchEntry& b = args.e[v];
    double* p = part + 2 * static_cast<int64_t>(v) * gridDim.x;
    const int mode = static_cast<int>(b.kind >> 3);
    if (mode == kWide || mode == kMixed) {
      if (b.kind & 2) {
        if (b.kind & 4)
          batch_item_wide<true, true, U, BMAX>(b, b.kind, p);
        else
          batch_item_wide<true, false, U, BMAX>(b, b.kind, p);
      } else {
        batch_item_wide<false, true, U, BMAX>(b, b.kind, p);
      }
    } else if (b.kind & 1) {
      batch_by_op<double, U, BMAX>(b, b.kind, p);
    } else {
      batch_by_op<float, U, BMAX>(b, b.kind, p);
    }
    __syncthreads();
  }
}

template <typename T>
__device__ __forceinline__ void batch_pass2_by_mode(const BatchEntry& b, const double2* pairs,
                                                    int nparts) {
  switch (static_cast<int>(b.kind >> 3)) {
    case kPlain: pass2_block<T, kPlain>(pairs, nparts, b.out, 0); break;
    case kFast: pass2_block<T, kFast>(pairs, nparts, b.out, 0); break;
    case kRigorous: pass2_block<T, kRigorous>(pairs, nparts, b.out, 0); break;
    case kKahan: pass2_block<T, kKahan>(pairs, nparts, b.out, 0); break;
    case kFastRounded: pass2_block<T, kFastRounded>(pairs, nparts, b.out, 0); break;
    case kRigorousRounded: pass2_block<T, kRigorousRounded>(pairs, nparts, b.out, 0); break;
    case kWide:
      if constexpr (sizeof(T) == 4)
        pass2_block<T, kWide>(pairs, nparts, b.out, 0);
      else
        pass2_block<T, kDoubleDouble>(pairs, nparts, b.out, 0);
      break;
    default:
      if constexpr (sizeof(T) == 4) pass2_block<T, kMixed>(pairs, nparts, b.out, 0);
      break;
  }
}

// Pass 2: block v combines item v's block pairs (step 7) and finalizes.
__global__ void __launch_bounds__(kPass2Lanes)
batch_pass2_kernel(const BatchArgs args, const double* __restrict__ part, int nparts) {
  const BatchEntry& b = args.e[blockIdx.x];
  const double2* pairs =
      reinterpret_cast<const double2*>(part) + static_cast<int64_t>(blockIdx.x) * nparts;
  if (b.kind & 1)
    batch_pass2_by_mode<double>(b, pairs, nparts);
  else
    batch_pass2_by_mode<float>(b, pairs, nparts);
}

}  // namespace twofold

using namespace twofold;
using namespace twofold::host;

namespace {

// Items that read at most this much each run side by side (one block set
// each), as in the multi-vector calls; otherwise one set walks them in turn.
constexpr int64_t kBatchSideBytes = int64_t(1) << 26;

bool batch_mode_ok(int dtype, bool dot, int mode) { return mode_ok(dtype, dot, mode); }

int64_t item_bytes(const twofold_batch_item_t& it) {
  return it.n * it.dtype * (it.is_dot ? 2 : 1);
}

// Checks every item; the launch is the single-vector one of the item that
// reads the most bytes (the first such), or the given one.
int resolve_batch(const twofold_batch_item_t* items, int64_t count,
                  const twofold_launch_t* launch, twofold_launch_t* lc, int64_t* max_bytes) {
  if (count < 0 || count > kMaxBatch || (count > 0 && !items)) return TWOFOLD_EINVAL;
  int64_t best = -1, bi = 0;
  for (int64_t v = 0; v < count; v++) {
    const twofold_batch_item_t& it = items[v];
    if (!valid_dtype(it.dtype) || !valid_count(it.n) || (it.is_dot != 0 && it.is_dot != 1) ||
        !batch_mode_ok(it.dtype, it.is_dot != 0, it.mode) || it.reserved != 0)
      return TWOFOLD_EINVAL;
    if (item_bytes(it) > best) {
      best = item_bytes(it);
      bi = v;
    }
  }
  *max_bytes = best < 0 ? 0 : best;
  if (count == 0) return TWOFOLD_OK;
  const twofold_batch_item_t& m = items[bi];
  const int rc = resolve_single(m.dtype, m.is_dot != 0, m.mode, m.n, launch, lc);
  // the batch kernel holds every form's code; its instance for blocks of
  // up to 1024 threads spills above four vectors a round, so a default
  // launch of such blocks takes at most four
  if (!rc && !launch && lc->unroll > 4 && lc->block_threads > kSmallBlock) lc->unroll = 4;
  return rc;
}

int launch_batch(const BatchArgs& a, int count, int sets, bool wide, const twofold_launch_t& lc,
                 double* part, hipStream_t st) {
  const dim3 grid(lc.grid_blocks, unsigned(sets)), block(lc.block_threads);
  const int rc = by_shape(lc, [&](auto u, auto bmax) {
    constexpr int U = decltype(u)::value, BMAX = decltype(bmax)::value;
    return wide ? launch_kernel(batch_kernel_wide<U, BMAX>, grid, block, st, a, count, part)
                : launch_kernel(batch_kernel<U, BMAX>, grid, block, st, a, count, part);
  });
  if (rc || lc.grid_blocks == 1) return rc;
  return launch_kernel(batch_pass2_kernel, dim3(unsigned(count)), dim3(kPass2Lanes), st, a, part,
                       lc.grid_blocks);
}

}  // namespace

extern "C" {

size_t twofold_workspace_bytes_batch(const twofold_batch_item_t* items, int64_t count,
                                     const twofold_launch_t* launch) {
  twofold_launch_t lc;
  int64_t mb = 0;
  if (resolve_batch(items, count, launch, &lc, &mb)) return 0;
  if (count == 0) return align256(16);
  return multi_ws_bytes(lc, count);
}

}  // extern "C"

namespace {

// The block pairs of twofold_batch_static: one array per device, in device
// memory for the life of the process. Host code never passes the array's
// name to a kernel (on the host it is only a stand-in): the address each
// device gives the array comes from hipGetSymbolAddress, looked up on the
// first call on that device and kept per device.
constexpr size_t kStaticScratchBytes = size_t(TWOFOLD_STATIC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// The current device's address of scratch (set up once per device).
int static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return TWOFOLD_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return TWOFOLD_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TWOFOLD_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TWOFOLD_OK;
}

// twofold_batch with its block pairs in ws, or (ws_static) in the device's
// static scratch.
int batch_common(const twofold_batch_item_t* items, int64_t count, const twofold_launch_t* launch,
                 void* ws, size_t ws_bytes, bool ws_static, void* stream) {
  twofold_launch_t lc;
  int64_t max_bytes = 0;
  const int rc = resolve_batch(items, count, launch, &lc, &max_bytes);
  if (rc) return rc;
  BatchArgs a;
  bool wide = false;  // any item with binary64 results: the kernel that holds them
  for (int64_t v = 0; v < count; v++) {
    const twofold_batch_item_t& it = items[v];
    const bool dot = it.is_dot != 0;
    // data pointers may be NULL only when there is no data
    if (!it.out || (!it.x && it.n > 0) || (dot && !it.y && it.n > 0)) return TWOFOLD_EINVAL;
    if (!elem_aligned(it.x, it.dtype) || (dot && !elem_aligned(it.y, it.dtype)) ||
        !elem_aligned(it.out, out_f64(it.dtype, it.mode) ? 8 : 4))
      return TWOFOLD_EALIGN;
    if (it.mode == kWide || it.mode == kMixed) wide = true;
    const bool yv = !dot || ((reinterpret_cast<uintptr_t>(it.y) -
                              reinterpret_cast<uintptr_t>(it.x)) & 15u) == 0;
    a.e[v].x = it.x;
    a.e[v].y = dot ? it.y : nullptr;
    a.e[v].out = it.out;
    a.e[v].n = it.n;
    a.e[v].kind = int64_t(it.dtype == 8) | (int64_t(dot) << 1) | (int64_t(yv) << 2) |
                  (int64_t(it.mode) << 3);
  }
  for (int64_t v = count; v < kMaxBatch; v++) a.e[v] = BatchEntry{nullptr, nullptr, nullptr, 0, 0};
  if (count == 0) return TWOFOLD_OK;
  if (ws_static) {
    if (lc.grid_blocks > 1 && multi_ws_bytes(lc, count) > kStaticScratchBytes)
      return TWOFOLD_EWORKSPACE;
    const int rs = static_scratch(&ws);
    if (rs) return rs;
  } else if (lc.grid_blocks > 1 && !ws_ok(ws, ws_bytes, multi_ws_bytes(lc, count))) {
    return TWOFOLD_EWORKSPACE;
  }
  const int sets = max_bytes <= kBatchSideBytes ? int(count) : 1;
  double* part = static_cast<double*>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launch_batch(a, int(count), sets, wide, lc, part, st);
}

}  // namespace

extern "C" {

int twofold_batch(const twofold_batch_item_t* items, int64_t count,
                  const twofold_launch_t* launch, void* ws, size_t ws_bytes, void* stream) {
  return batch_common(items, count, launch, ws, ws_bytes, false, stream);
}

int twofold_batch_static(const twofold_batch_item_t* items, int64_t count,
                         const twofold_launch_t* launch, void* stream) {
  return batch_common(items, count, launch, nullptr, 0, true, stream);
}

}  // extern "C"
