// twofold.hip: host side of the single-vector entry points of
// include/twofold.h, plus the launch and status queries.
//
// Argument checks run on the host before any HIP call; launches go to the
// caller's stream; nothing here allocates, frees or synchronises, so every
// call can be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "host_common.hpp"
#include "kernels.hpp"
#include "twofold.h"

using namespace twofold;
using namespace twofold::host;

namespace {

template <typename T, typename A, int M, bool DOT, bool YV>
int launch_single_u(const T* x, const T* y, int64_t n, const twofold_launch_t& lc, double* part,
                    void* out, hipStream_t st) {
  const dim3 grid(lc.grid_blocks), block(lc.block_threads);
  const int rc = by_shape(lc, [&](auto u, auto bmax) {
    return launch_kernel(single_kernel<T, A, M, DOT, YV, decltype(u)::value, decltype(bmax)::value>,
                         grid, block, st, x, y, n, part, out);
  });
  if (rc || lc.grid_blocks == 1) return rc;
  return launch_kernel(single_pass2_kernel<T, M>, dim3(1), dim3(kPass2Lanes), st, part,
                       lc.grid_blocks, out);
}

template <typename T, typename A, int M, bool DOT>
int launch_single(const T* x, const T* y, int64_t n, const twofold_launch_t& lc, double* part,
                  void* out, hipStream_t st) {
  if constexpr (DOT) {
    if (!y_vector_ok(x, y)) return launch_single_u<T, A, M, DOT, false>(x, y, n, lc, part, out, st);
  }
  return launch_single_u<T, A, M, DOT, true>(x, y, n, lc, part, out, st);
}

template <typename T, bool DOT>
int single_by_mode(int mode, const T* x, const T* y, int64_t n, const twofold_launch_t& lc,
                   double* part, void* out, hipStream_t st) {
  switch (mode) {
    case kPlain: return launch_single<T, T, kPlain, DOT>(x, y, n, lc, part, out, st);
    case kFast: return launch_single<T, T, kFast, DOT>(x, y, n, lc, part, out, st);
    case kRigorous: return launch_single<T, T, kRigorous, DOT>(x, y, n, lc, part, out, st);
    case kKahan: return launch_single<T, T, kKahan, DOT>(x, y, n, lc, part, out, st);
    case kFastRounded:
      if constexpr (DOT) return launch_single<T, T, kFastRounded, DOT>(x, y, n, lc, part, out, st);
      return TWOFOLD_EINVAL;
    case kRigorousRounded:
      if constexpr (DOT) return launch_single<T, T, kRigorousRounded, DOT>(x, y, n, lc, part, out, st);
      return TWOFOLD_EINVAL;
    case kWide:
      if constexpr (sizeof(T) == 4)
        return launch_single<T, double, kWide, DOT>(x, y, n, lc, part, out, st);
      else
        return launch_single<T, double, kDoubleDouble, DOT>(x, y, n, lc, part, out, st);
    case kMixed:
      if constexpr (sizeof(T) == 4) return launch_single<T, double, kMixed, DOT>(x, y, n, lc, part, out, st);
      return TWOFOLD_EINVAL;
    default: return TWOFOLD_EINVAL;
  }
}

// Common body of the single-vector entry points.
template <typename T, bool DOT>
int single_entry(const T* x, const T* y, int64_t n, int mode, const twofold_launch_t* launch,
                 void* out, void* ws, size_t ws_bytes, void* stream) {
  const int dtype = int(sizeof(T));
  // Data pointers may be NULL only when there is no data (torch hands out
  // NULL for empty tensors).
  if ((!x && n > 0) || !out || (DOT && !y && n > 0) || !valid_count(n)) return TWOFOLD_EINVAL;
  if (!mode_ok(dtype, DOT, mode)) return TWOFOLD_EINVAL;
  if (!elem_aligned(x, dtype) || (DOT && !elem_aligned(y, dtype))) return TWOFOLD_EALIGN;
  if (!elem_aligned(out, out_f64(dtype, mode) ? 8 : 4)) return TWOFOLD_EALIGN;
  twofold_launch_t lc;
  const int rc = resolve_single(dtype, DOT, mode, n, launch, &lc);
  if (rc) return rc;
  if (lc.grid_blocks > 1 && !ws_ok(ws, ws_bytes, single_ws_bytes(lc))) return TWOFOLD_EWORKSPACE;
  return single_by_mode<T, DOT>(mode, x, y, n, lc, static_cast<double*>(ws), out,
                                static_cast<hipStream_t>(stream));
}

// ---- several vectors in one launch ------------------------------------------
template <typename T, typename A, int M, bool DOT, bool YV>
int launch_multi_u(const MultiArgs<T>& a, int64_t count, int sets, const twofold_launch_t& lc,
                   double* part, void* out, hipStream_t st) {
  const dim3 grid(lc.grid_blocks, unsigned(sets)), block(lc.block_threads);
  const int c = int(count);
  const int rc = by_shape(lc, [&](auto u, auto bmax) {
    return launch_kernel(multi_kernel<T, A, M, DOT, YV, decltype(u)::value, decltype(bmax)::value>,
                         grid, block, st, a, c, part, out);
  });
  if (rc || lc.grid_blocks == 1) return rc;
  return launch_kernel(single_pass2_kernel<T, M>, dim3(unsigned(count)), dim3(kPass2Lanes), st,
                       part, lc.grid_blocks, out);
}

template <typename T, typename A, int M, bool DOT>
int launch_multi(const MultiArgs<T>& a, int64_t count, int sets, bool yv,
                 const twofold_launch_t& lc, double* part, void* out, hipStream_t st) {
  if constexpr (DOT) {
    if (!yv) return launch_multi_u<T, A, M, DOT, false>(a, count, sets, lc, part, out, st);
  }
  return launch_multi_u<T, A, M, DOT, true>(a, count, sets, lc, part, out, st);
}

template <typename T, bool DOT>
int multi_by_mode(int mode, const MultiArgs<T>& a, int64_t count, int sets, bool yv,
                  const twofold_launch_t& lc, double* part, void* out, hipStream_t st) {
  switch (mode) {
    case kPlain: return launch_multi<T, T, kPlain, DOT>(a, count, sets, yv, lc, part, out, st);
    case kFast: return launch_multi<T, T, kFast, DOT>(a, count, sets, yv, lc, part, out, st);
    case kRigorous: return launch_multi<T, T, kRigorous, DOT>(a, count, sets, yv, lc, part, out, st);
    case kKahan: return launch_multi<T, T, kKahan, DOT>(a, count, sets, yv, lc, part, out, st);
    case kFastRounded:
      if constexpr (DOT) return launch_multi<T, T, kFastRounded, DOT>(a, count, sets, yv, lc, part, out, st);
      return TWOFOLD_EINVAL;
    case kRigorousRounded:
      if constexpr (DOT)
        return launch_multi<T, T, kRigorousRounded, DOT>(a, count, sets, yv, lc, part, out, st);
      return TWOFOLD_EINVAL;
    case kWide:
      if constexpr (sizeof(T) == 4)
        return launch_multi<T, double, kWide, DOT>(a, count, sets, yv, lc, part, out, st);
      else
        return launch_multi<T, double, kDoubleDouble, DOT>(a, count, sets, yv, lc, part, out, st);
    case kMixed:
      if constexpr (sizeof(T) == 4)
        return launch_multi<T, double, kMixed, DOT>(a, count, sets, yv, lc, part, out, st);
      return TWOFOLD_EINVAL;
    default: return TWOFOLD_EINVAL;
  }
}

// Block sets of a multi-vector launch (the result does not depend on it):
// when no vector reads more than kMultiSideBytes, the vectors run side by
// side, one set each, so short vectors overlap their latencies; longer
// ones go one after another through a single set, which then streams them
// like one long vector. Measured on six to 64 dots: side by side is up to
// 3.8 times faster for small vectors and even at 64 MiB per vector; one
// set is 1-3% faster at 128-256 MiB per vector.
constexpr int64_t kMultiSideBytes = int64_t(1) << 26;

int multi_sets(int64_t count, int64_t nmax, int dtype, bool is_dot) {
  return nmax * dtype * (is_dot ? 2 : 1) <= kMultiSideBytes ? int(count) : 1;
}

// The launch of a multi-vector call: the single-vector one for the longest
// vector (or the given one).
int resolve_multi(int dtype, bool is_dot, int mode, const int64_t* n, int64_t count,
                  const twofold_launch_t* launch, twofold_launch_t* lc) {
  int64_t nmax = 0;
  for (int64_t v = 0; v < count; v++) nmax = n[v] > nmax ? n[v] : nmax;
  return resolve_single(dtype, is_dot, mode, nmax, launch, lc);
}

template <typename T, bool DOT>
int multi_entry(const T* const* x, const T* const* y, const int64_t* n, int64_t count, int mode,
                const twofold_launch_t* launch, void* out, void* ws, size_t ws_bytes,
                void* stream) {
  const int dtype = int(sizeof(T));
  if (count < 0 || count > kMaxMulti || !out) return TWOFOLD_EINVAL;
  if (count > 0 && (!x || !n || (DOT && !y))) return TWOFOLD_EINVAL;
  if (!mode_ok(dtype, DOT, mode)) return TWOFOLD_EINVAL;
  if (!elem_aligned(out, out_f64(dtype, mode) ? 8 : 4)) return TWOFOLD_EALIGN;
  MultiArgs<T> a;
  bool yv = true;
  int64_t nmax = 0;
  for (int64_t v = 0; v < count; v++) {
    if (!valid_count(n[v]) || (!x[v] && n[v] > 0) || (DOT && !y[v] && n[v] > 0))
      return TWOFOLD_EINVAL;
    if (!elem_aligned(x[v], dtype) || (DOT && !elem_aligned(y[v], dtype))) return TWOFOLD_EALIGN;
    a.x[v] = x[v];
    a.y[v] = DOT ? y[v] : nullptr;
    a.n[v] = n[v];
    nmax = n[v] > nmax ? n[v] : nmax;
    if (DOT && !y_vector_ok(x[v], y[v])) yv = false;
  }
  for (int64_t v = count; v < kMaxMulti; v++) {
    a.x[v] = nullptr;
    a.y[v] = nullptr;
    a.n[v] = 0;
  }
  if (count == 0) return TWOFOLD_OK;
  twofold_launch_t lc;
  const int rc = resolve_multi(dtype, DOT, mode, n, count, launch, &lc);
  if (rc) return rc;
  if (lc.grid_blocks > 1 && !ws_ok(ws, ws_bytes, multi_ws_bytes(lc, count)))
    return TWOFOLD_EWORKSPACE;
  return multi_by_mode<T, DOT>(mode, a, count, multi_sets(count, nmax, dtype, DOT), yv, lc,
                               static_cast<double*>(ws), out, static_cast<hipStream_t>(stream));
}

}  // namespace

extern "C" {

int twofold_default_launch(int kind, int dtype, int is_dot, int mode, int64_t n, int64_t nseg,
                           twofold_launch_t* out) {
  if (!out || !valid_dtype(dtype) || (kind != 0 && kind != 1) || !valid_count(n) ||
      !valid_count(nseg))
    return TWOFOLD_EINVAL;
  if (!mode_ok(dtype, is_dot != 0, mode)) return TWOFOLD_EINVAL;
  if (kind == 0) return resolve_single(dtype, is_dot != 0, mode, n, nullptr, out);
  return resolve_seg(dtype, is_dot != 0, mode, n, nseg, nullptr, out);
}

int twofold_tuned_launch(int kind, int dtype, int is_dot, int mode, int64_t n, int64_t nseg,
                         twofold_launch_t* out) {
  const int rc = twofold_default_launch(kind, dtype, is_dot, mode, n, nseg, out);
  if (rc) return rc;
  twofold_launch_t row;
  const int64_t len = kind == 1 ? mean_len(n, nseg) : 0;
  return lookup_rows(kind, dtype, is_dot != 0, mode, n, len, &row) ? TWOFOLD_OK : TWOFOLD_ENOTUNED;
}

size_t twofold_workspace_bytes_single(int dtype, int is_dot, int mode, int64_t n,
                                      const twofold_launch_t* launch) {
  if (!valid_dtype(dtype) || !valid_count(n) || !mode_ok(dtype, is_dot != 0, mode)) return 0;
  twofold_launch_t lc;
  if (resolve_single(dtype, is_dot != 0, mode, n, launch, &lc)) return 0;
  return single_ws_bytes(lc);
}

int twofold_sum_f32(const float* x, int64_t n, int mode, const twofold_launch_t* launch,
                    twofold_f32_t* out, void* ws, size_t ws_bytes, void* stream) {
  // binary64 results: twofold_sumd_f32, twofold_sum_mixed_f32
  if (mode == kWide || mode == kMixed) return TWOFOLD_EINVAL;
  return single_entry<float, false>(x, nullptr, n, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_sum_f64(const double* x, int64_t n, int mode, const twofold_launch_t* launch,
                    twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream) {
  if (mode == kWide) return TWOFOLD_EINVAL;  // the wider accumulator: twofold_sumd_f64
  return single_entry<double, false>(x, nullptr, n, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_dot_f32(const float* x, const float* y, int64_t n, int mode,
                    const twofold_launch_t* launch, twofold_f32_t* out, void* ws, size_t ws_bytes,
                    void* stream) {
  // binary64 results: twofold_dotd_f32, twofold_dot_mixed_f32
  if (mode == kWide || mode == kMixed) return TWOFOLD_EINVAL;
  return single_entry<float, true>(x, y, n, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_dot_f64(const double* x, const double* y, int64_t n, int mode,
                    const twofold_launch_t* launch, twofold_f64_t* out, void* ws, size_t ws_bytes,
                    void* stream) {
  if (mode == kWide) return TWOFOLD_EINVAL;  // the wider accumulator: twofold_dotd_f64
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
int twofold_sum_mixed_f32(const float* x, int64_t n, const twofold_launch_t* launch,
                          twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream) {
  return single_entry<float, false>(x, nullptr, n, kMixed, launch, out, ws, ws_bytes, stream);
}
int twofold_dot_mixed_f32(const float* x, const float* y, int64_t n,
                          const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                          size_t ws_bytes, void* stream) {
  return single_entry<float, true>(x, y, n, kMixed, launch, out, ws, ws_bytes, stream);
}
int twofold_sumd_f64(const double* x, int64_t n, const twofold_launch_t* launch,
                     twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream) {
  return single_entry<double, false>(x, nullptr, n, kWide, launch, out, ws, ws_bytes, stream);
}
int twofold_dotd_f64(const double* x, const double* y, int64_t n, const twofold_launch_t* launch,
                     twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream) {
  return single_entry<double, true>(x, y, n, kWide, launch, out, ws, ws_bytes, stream);
}

size_t twofold_workspace_bytes_multi(int dtype, int is_dot, int mode, const int64_t* n,
                                     int64_t count, const twofold_launch_t* launch) {
  if (!valid_dtype(dtype) || count < 0 || count > kMaxMulti || (count > 0 && !n) ||
      !mode_ok(dtype, is_dot != 0, mode))
    return 0;
  for (int64_t v = 0; v < count; v++)
    if (!valid_count(n[v])) return 0;
  twofold_launch_t lc;
  if (resolve_multi(dtype, is_dot != 0, mode, n, count, launch, &lc)) return 0;
  return multi_ws_bytes(lc, count);
}

int twofold_multisum_f32(const float* const* x, const int64_t* n, int64_t count, int mode,
                         const twofold_launch_t* launch, twofold_f32_t* out, void* ws,
                         size_t ws_bytes, void* stream) {
  // binary64 results: twofold_multisumd_f32, twofold_multisum_mixed_f32
  if (mode == kWide || mode == kMixed) return TWOFOLD_EINVAL;
  return multi_entry<float, false>(x, nullptr, n, count, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_multisum_f64(const double* const* x, const int64_t* n, int64_t count, int mode,
                         const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                         size_t ws_bytes, void* stream) {
  if (mode == kWide) return TWOFOLD_EINVAL;  // the wider accumulator: twofold_multisumd_f64
  return multi_entry<double, false>(x, nullptr, n, count, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_multidot_f32(const float* const* x, const float* const* y, const int64_t* n,
                         int64_t count, int mode, const twofold_launch_t* launch,
                         twofold_f32_t* out, void* ws, size_t ws_bytes, void* stream) {
  // binary64 results: twofold_multidotd_f32, twofold_multidot_mixed_f32
  if (mode == kWide || mode == kMixed) return TWOFOLD_EINVAL;
  return multi_entry<float, true>(x, y, n, count, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_multidot_f64(const double* const* x, const double* const* y, const int64_t* n,
                         int64_t count, int mode, const twofold_launch_t* launch,
                         twofold_f64_t* out, void* ws, size_t ws_bytes, void* stream) {
  if (mode == kWide) return TWOFOLD_EINVAL;  // the wider accumulator: twofold_multidotd_f64
  return multi_entry<double, true>(x, y, n, count, mode, launch, out, ws, ws_bytes, stream);
}
int twofold_multisumd_f32(const float* const* x, const int64_t* n, int64_t count,
                          const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                          size_t ws_bytes, void* stream) {
  return multi_entry<float, false>(x, nullptr, n, count, kWide, launch, out, ws, ws_bytes, stream);
}
int twofold_multisumd_f64(const double* const* x, const int64_t* n, int64_t count,
                          const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                          size_t ws_bytes, void* stream) {
  return multi_entry<double, false>(x, nullptr, n, count, kWide, launch, out, ws, ws_bytes, stream);
}
int twofold_multidotd_f32(const float* const* x, const float* const* y, const int64_t* n,
                          int64_t count, const twofold_launch_t* launch, twofold_f64_t* out,
                          void* ws, size_t ws_bytes, void* stream) {
  return multi_entry<float, true>(x, y, n, count, kWide, launch, out, ws, ws_bytes, stream);
}
int twofold_multidotd_f64(const double* const* x, const double* const* y, const int64_t* n,
                          int64_t count, const twofold_launch_t* launch, twofold_f64_t* out,
                          void* ws, size_t ws_bytes, void* stream) {
  return multi_entry<double, true>(x, y, n, count, kWide, launch, out, ws, ws_bytes, stream);
}
int twofold_multisum_mixed_f32(const float* const* x, const int64_t* n, int64_t count,
                               const twofold_launch_t* launch, twofold_f64_t* out, void* ws,
                               size_t ws_bytes, void* stream) {
  return multi_entry<float, false>(x, nullptr, n, count, kMixed, launch, out, ws, ws_bytes, stream);
}
int twofold_multidot_mixed_f32(const float* const* x, const float* const* y, const int64_t* n,
                               int64_t count, const twofold_launch_t* launch, twofold_f64_t* out,
                               void* ws, size_t ws_bytes, void* stream) {
  return multi_entry<float, true>(x, y, n, count, kMixed, launch, out, ws, ws_bytes, stream);
}

const char* twofold_strerror(int status) {
  switch (status) {
    case TWOFOLD_OK: return "ok";
    case TWOFOLD_EINVAL: return "invalid argument";
    case TWOFOLD_EWORKSPACE: return "workspace missing, misaligned or too small";
    case TWOFOLD_EHIP: return "HIP runtime error";
    case TWOFOLD_EALIGN: return "data pointer not aligned to its element size";
    case TWOFOLD_EOFFSETS: return "segment offsets must start at 0 and not decrease";
    case TWOFOLD_ENOTUNED: return "no measured launch for this configuration (default borrowed)";
    case TWOFOLD_ECAPTURE: return "not allowed while a stream capture is under way";
    default: return "unknown status";
  }
}

}  // extern "C"
