// probes.hip: the measuring instruments of the library, gfx950 versions of
// the paper's read1/read2 memory-only functions (section "Memory reading")
// and its p-functions that compute without reading memory (section "Purely
// computing"). They bound the reduction kernels from above: the read probe
// gives the achievable HBM stream rate, the compute probe the ALU rate of
// each summation step when no data has to be fetched.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "eft.hpp"
#include "twofold.h"

using namespace twofold;

namespace {

// Stream one or two arrays with 16-byte non-temporal loads (the load the
// reduction kernels use) in the single-vector lane order and fold every
// loaded bit into one word, so no load is dead code.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 load_nt16(const uint4* p) {
  const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

template <bool TWO, int U>
__global__ void __launch_bounds__(1024)
read_probe_kernel(const uint4* __restrict__ x, const uint4* __restrict__ y, int64_t nvec,
                  uint64_t* __restrict__ sink) {
  const int64_t L = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  const int64_t per_round = int64_t(U) * L;
  const int64_t full = nvec / per_round;
  int64_t k0 = g;
  for (int64_t q = 0; q < full; q++, k0 += per_round) {
    uint4 a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; u++) a[u] = load_nt16(x + k0 + u * L);
    if constexpr (TWO) {
#pragma unroll
      for (int u = 0; u < U; u++) b[u] = load_nt16(y + k0 + u * L);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      acc |= a[u].x | a[u].y | a[u].z | a[u].w;
      if constexpr (TWO) acc |= b[u].x | b[u].y | b[u].z | b[u].w;
    }
  }
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int64_t k = k0 + u * L;
    if (k < nvec) {
      const uint4 a = load_nt16(x + k);
      acc |= a.x | a.y | a.z | a.w;
      if constexpr (TWO) {
        const uint4 b = load_nt16(y + k);
        acc |= b.x | b.y | b.z | b.w;
      }
    }
  }
  // One word per block: OR across the block through LDS.
  __shared__ uint32_t sh[16];
  for (int d = 1; d < 64; d <<= 1) acc |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(acc), d));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
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
  compute_probe_kernel<T, A, M, DOT, 4><<<dim3(lc.grid_blocks), dim3(lc.block_threads), 0, st>>>(
      static_cast<const T*>(seed), iters, sink);
  return hipGetLastError() == hipSuccess ? TWOFOLD_OK : TWOFOLD_EHIP;
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
  if (!x || !sink || nbytes < 0 || nbytes % 16 || !launch_ok(launch)) return TWOFOLD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(x) & 15u) || (y && (reinterpret_cast<uintptr_t>(y) & 15u)) ||
      (reinterpret_cast<uintptr_t>(sink) & 7u))
    return TWOFOLD_EALIGN;
  const int64_t nvec = nbytes / 16;
  const dim3 grid(launch->grid_blocks), block(launch->block_threads);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint4* xv = static_cast<const uint4*>(x);
  const uint4* yv = static_cast<const uint4*>(y);
#define TWOFOLD_READ(TWO, UU) read_probe_kernel<TWO, UU><<<grid, block, 0, st>>>(xv, yv, nvec, sink)
  const int u = launch->unroll;
  if (y) {
    if (u == 1) TWOFOLD_READ(true, 1); else if (u == 2) TWOFOLD_READ(true, 2);
    else if (u == 4) TWOFOLD_READ(true, 4); else if (u == 8) TWOFOLD_READ(true, 8);
    else return TWOFOLD_EINVAL;
  } else {
    if (u == 1) TWOFOLD_READ(false, 1); else if (u == 2) TWOFOLD_READ(false, 2);
    else if (u == 4) TWOFOLD_READ(false, 4); else if (u == 8) TWOFOLD_READ(false, 8);
    else return TWOFOLD_EINVAL;
  }
#undef TWOFOLD_READ
  return hipGetLastError() == hipSuccess ? TWOFOLD_OK : TWOFOLD_EHIP;
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
