// probes.hip: the measuring instruments of the library, gfx950 versions of
// the paper's read1/read2 memory-only functions (section "Memory reading")
// and its p-functions that compute without reading memory (section "Purely
// computing").
//
// The read probe runs the single-vector kernel's own lane loop (lane_reduce:
// the same 16-byte non-temporal loads in the same lane order, the same
// loads one round ahead, the same register budget per block size) with the
// summation step replaced by a bit-OR of the loaded words, so it measures
// what that loop can stream when no arithmetic has to keep up. The compute
// probe runs each form's step on register-resident items, with no memory
// traffic: the ALU rate of each summation step.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "host_common.hpp"
#include "kernels.hpp"
#include "twofold.h"

using namespace twofold;
using namespace twofold::host;

namespace {

// One or two arrays of binary32 words (n words each, 16-byte aligned, n a
// multiple of 4) in the single-vector lane order of the launch; each block
// writes the OR of every word its lanes loaded to sink[block].
template <bool TWO, int U, int BMAX>
__global__ void __launch_bounds__(BMAX)
read_probe_kernel(const float* __restrict__ x, const float* __restrict__ y, int64_t n,
                  uint64_t* __restrict__ sink) {
  const int64_t L = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  float s, e;
  lane_reduce<float, float, kProbeOr, TWO, true, U, rounds_ahead_single<BMAX, TWO, U>()>(
      x, y, n, 0, L, g, s, e);
  wave_combine<kProbeOr>(s, e);
  __shared__ uint32_t sh[16];
  if ((threadIdx.x & 63) == kWaveRoot) sh[threadIdx.x >> 6] = __float_as_uint(s);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = 0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); w++) r |= sh[w];
    sink[blockIdx.x] = r;
  }
}

// The summation step of each mode applied to register-resident items: the
// U*W items are loaded once; every iteration feeds all of them through the
// lane's W chains again, the whole step included (a dot's product and
// remainder too). The chains' results go to sink so nothing is dead.
template <typename T, typename A, int M, bool DOT, int U>
__global__ void __launch_bounds__(1024)
compute_probe_kernel(const T* __restrict__ seed, int64_t iters, double* __restrict__ sink) {
  constexpr int W = 16 / static_cast<int>(sizeof(T));
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  T xv[U][W], yv[U][W];
#pragma unroll
  for (int u = 0; u < U; u++)
#pragma unroll
    for (int j = 0; j < W; j++) {
      xv[u][j] = seed[(u * W + j) & 63];
      yv[u][j] = seed[(u * W + j + 17) & 63];
    }
  A cs[W], ce[W];
#pragma unroll
  for (int j = 0; j < W; j++) {
    cs[j] = static_cast<A>(seed[j]) * static_cast<A>(g & 7);
    ce[j] = A(0);
  }
  for (int64_t it = 0; it < iters; it++) {
    // An empty register barrier: the compiler must assume the items changed,
    // so the per-item work (products, FMA remainders) stays in the loop
    // instead of being hoisted out of it. It emits no instruction.
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int j = 0; j < W; j++) {
        asm volatile("" : "+v"(xv[u][j]));
        if constexpr (DOT) asm volatile("" : "+v"(yv[u][j]));
      }
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int j = 0; j < W; j++) step<M, DOT>(cs[j], ce[j], xv[u][j], yv[u][j]);
  }
  A s = cs[0], e = ce[0];
#pragma unroll
  for (int j = 1; j < W; j++) combine<M>(s, e, cs[j], ce[j]);
  sink[2 * g] = static_cast<double>(s);
  sink[2 * g + 1] = static_cast<double>(e);
}

template <typename T, typename A, int M, bool DOT>
int launch_compute(const void* seed, int64_t iters, const twofold_launch_t& lc, double* sink,
                   hipStream_t st) {
  return launch_kernel(compute_probe_kernel<T, A, M, DOT, 4>, dim3(lc.grid_blocks),
                       dim3(lc.block_threads), st, static_cast<const T*>(seed), iters, sink);
}

template <typename T, bool DOT>
int compute_by_mode(int mode, const void* seed, int64_t iters, const twofold_launch_t& lc,
                    double* sink, hipStream_t st) {
  switch (mode) {
    case kPlain: return launch_compute<T, T, kPlain, DOT>(seed, iters, lc, sink, st);
    case kFast: return launch_compute<T, T, kFast, DOT>(seed, iters, lc, sink, st);
    case kRigorous: return launch_compute<T, T, kRigorous, DOT>(seed, iters, lc, sink, st);
    case kKahan: return launch_compute<T, T, kKahan, DOT>(seed, iters, lc, sink, st);
    case kFastRounded:
      if constexpr (DOT) return launch_compute<T, T, kFastRounded, DOT>(seed, iters, lc, sink, st);
      return TWOFOLD_EINVAL;
    case kRigorousRounded:
      if constexpr (DOT) return launch_compute<T, T, kRigorousRounded, DOT>(seed, iters, lc, sink, st);
      return TWOFOLD_EINVAL;
    case kWide:
      if constexpr (sizeof(T) == 4)
        return launch_compute<T, double, kWide, DOT>(seed, iters, lc, sink, st);
      else
        return launch_compute<T, double, kDoubleDouble, DOT>(seed, iters, lc, sink, st);
    case kMixed:
      if constexpr (sizeof(T) == 4)
        return launch_compute<T, double, kMixed, DOT>(seed, iters, lc, sink, st);
      return TWOFOLD_EINVAL;
    default: return TWOFOLD_EINVAL;
  }
}

bool launch_ok(const twofold_launch_t* lc) {
  return lc && lc->block_threads >= 64 && lc->block_threads <= 1024 && lc->block_threads % 64 == 0 &&
         lc->grid_blocks >= 1 && lc->grid_blocks <= (1 << 20) && lc->reserved == 0;
}

}  // namespace

extern "C" {

int twofold_probe_read(const void* x, const void* y, int64_t nbytes, const twofold_launch_t* launch,
                       uint64_t* sink, void* stream) {
  if (!x || !sink || nbytes < 0 || nbytes % 16 || !launch_ok(launch) ||
      !valid_unroll(launch->unroll))
    return TWOFOLD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(x) & 15u) || (y && (reinterpret_cast<uintptr_t>(y) & 15u)) ||
      (reinterpret_cast<uintptr_t>(sink) & 7u))
    return TWOFOLD_EALIGN;
  const int64_t n = nbytes / 4;
  const dim3 grid(launch->grid_blocks), block(launch->block_threads);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const float* xf = static_cast<const float*>(x);
  const float* yf = static_cast<const float*>(y);
  return by_shape(*launch, [&](auto u, auto bmax) {
    constexpr int U = decltype(u)::value, BMAX = decltype(bmax)::value;
    return y ? launch_kernel(read_probe_kernel<true, U, BMAX>, grid, block, st, xf, yf, n, sink)
             : launch_kernel(read_probe_kernel<false, U, BMAX>, grid, block, st, xf, yf, n, sink);
  });
}

int twofold_probe_compute(int dtype, int is_dot, int mode, const void* seed, int64_t iters,
                          const twofold_launch_t* launch, double* sink, void* stream) {
  if (!seed || !sink || iters < 0 || !launch_ok(launch)) return TWOFOLD_EINVAL;
  if (dtype != 4 && dtype != 8) return TWOFOLD_EINVAL;
  if (mode < kPlain || mode > kMixed ||
      ((mode == kFastRounded || mode == kRigorousRounded) && !is_dot) ||
      (mode == kMixed && dtype != 4))
    return TWOFOLD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(seed) % uintptr_t(dtype)) || (reinterpret_cast<uintptr_t>(sink) & 7u))
    return TWOFOLD_EALIGN;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == 4)
    return is_dot ? compute_by_mode<float, true>(mode, seed, iters, *launch, sink, st)
                  : compute_by_mode<float, false>(mode, seed, iters, *launch, sink, st);
  return is_dot ? compute_by_mode<double, true>(mode, seed, iters, *launch, sink, st)
                : compute_by_mode<double, false>(mode, seed, iters, *launch, sink, st);
}

}  // extern "C"
