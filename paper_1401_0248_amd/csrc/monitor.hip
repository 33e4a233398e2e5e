// monitor.hip: the precision monitor of include/twofold.h. The paper
// suggests stopping a computation whose error term grows too large, as a
// sign that the precision in use is not enough ("Algorithms", the remarks
// after the rigorous form), and expects twofold summation to work for
// N below 1/u ("Overview"). This kernel turns both into per-result flags
// for a batch of results already on the device.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "host_common.hpp"
#include "twofold.h"

using namespace twofold::host;

namespace {

__global__ void zero_count_kernel(unsigned long long* c) { *c = 0ull; }

// One result per thread, grid-stride. Pairs are widened exactly to binary64
// and compared there; the count of nonzero flags is summed per wave and
// added once per wave (integer addition: the total does not depend on the
// order of the additions).
template <typename T>
__global__ void __launch_bounds__(256)
monitor_kernel(const T* __restrict__ pairs, int64_t count, const int64_t* __restrict__ off,
               int64_t n, double tau, int64_t inv_u, uint32_t* __restrict__ flags,
               unsigned long long* __restrict__ nflagged) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  unsigned int local = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += stride) {
    const double v = static_cast<double>(pairs[2 * i]);
    const double e = static_cast<double>(pairs[2 * i + 1]);
    const int64_t len = off ? off[i + 1] - off[i] : n;
    uint32_t f = 0;
    if (!__builtin_isfinite(v) || !__builtin_isfinite(e))
      f |= TWOFOLD_FLAG_NONFINITE;
    else if (__builtin_fabs(e) > tau * __builtin_fabs(v))
      f |= TWOFOLD_FLAG_ERROR;
    if (len >= inv_u) f |= TWOFOLD_FLAG_LENGTH;
    flags[i] = f;
    local += (f != 0u);
  }
  for (int d = 32; d >= 1; d >>= 1) local += __shfl_xor(local, d, 64);
  if ((threadIdx.x & 63) == 0 && local) atomicAdd(nflagged, static_cast<unsigned long long>(local));
}

}  // namespace

extern "C" {

int twofold_monitor(int dtype, const void* pairs, int64_t count, const int64_t* offsets, int64_t n,
                    double tau, uint32_t* flags, int64_t* nflagged, void* stream) {
  if (!valid_dtype(dtype) || count < 0 || !nflagged) return TWOFOLD_EINVAL;
  if (count > 0 && (!pairs || !flags)) return TWOFOLD_EINVAL;
  if (!offsets && n < 0) return TWOFOLD_EINVAL;
  if (!(tau >= 0.0) || tau > 1.7976931348623157e308) return TWOFOLD_EINVAL;  // NaN, Inf
  if (!elem_aligned(pairs, dtype) || !elem_aligned(offsets, 8) || !elem_aligned(flags, 4) ||
      !elem_aligned(nflagged, 8))
    return TWOFOLD_EALIGN;
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(nflagged);
  const int rc = launch_kernel(zero_count_kernel, dim3(1), dim3(1), st, cnt);
  if (rc || count == 0) return rc;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  const int64_t inv_u = dtype == 4 ? (int64_t(1) << 24) : (int64_t(1) << 53);
  if (dtype == 4)
    return launch_kernel(monitor_kernel<float>, dim3(unsigned(blocks)), dim3(256), st,
                         static_cast<const float*>(pairs), count, offsets, n, tau, inv_u, flags,
                         cnt);
  return launch_kernel(monitor_kernel<double>, dim3(unsigned(blocks)), dim3(256), st,
                       static_cast<const double*>(pairs), count, offsets, n, tau, inv_u, flags,
                       cnt);
}

}  // extern "C"
