// Internal helpers shared by the gplens translation units: error reporting,
// workspace carving, launch checks and small device utilities.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>

#include "../../include/gplens.h"

namespace gpl {

// Last error text, per host thread.
void set_error(const char* fmt, ...);
const char* last_error();

#define GPL_REQUIRE(cond, ...)              \
  do {                                      \
    if (!(cond)) {                          \
      ::gpl::set_error(__VA_ARGS__);        \
      return GPL_EINVAL;                    \
    }                                       \
  } while (0)

#define GPL_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      ::gpl::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call, hipGetErrorString(e_));    \
      return GPL_EHIP;                                                                       \
    }                                                                                        \
  } while (0)

#define GPL_LAUNCH_CHECK() GPL_HIP(hipGetLastError())

#define GPL_TRY(expr)     \
  do {                    \
    int rc_ = (expr);     \
    if (rc_ != GPL_OK) return rc_; \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }
__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }
__host__ __device__ inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Bump allocator over a caller-provided workspace. `take` returns nullptr when
// the workspace is exhausted (callers check `ok()` once after carving).
struct Carver {
  char* base;
  size_t cap;
  size_t used = 0;
  bool overflow = false;
  Carver(void* ws, size_t bytes) : base(static_cast<char*>(ws)), cap(bytes) {}
  template <class T>
  T* take(size_t count) {
    size_t off = align_up(used);
    size_t need = off + align_up(count * sizeof(T));
    if (base == nullptr || need > cap) {
      overflow = true;
      used = need;
      return nullptr;
    }
    used = need;
    return reinterpret_cast<T*>(base + off);
  }
  bool ok() const { return !overflow; }
};

// Size-only pass of the same carving sequence.
struct Sizer {
  size_t used = 0;
  template <class T>
  T* take(size_t count) {
    used = align_up(used) + align_up(count * sizeof(T));
    return nullptr;
  }
};

inline int check_ws(void* ws, size_t have, size_t need) {
  if (need == 0) return GPL_OK;
  if (ws == nullptr || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) {
    set_error("workspace must be non-NULL and %zu-byte aligned", kAlign);
    return GPL_EWORKSPACE;
  }
  if (have < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", have, need);
    return GPL_EWORKSPACE;
  }
  return GPL_OK;
}

// ---- device helpers

__device__ inline float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

template <class T>
__device__ inline T warp_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of p[0, cnt) over the 64 lanes of one wave in a fixed order (lane-strided
// partial sums, then a butterfly); the result is the same in every lane.
__device__ inline double wave_fold_sum(const double* __restrict__ p, int cnt) {
  double s = 0.0;
  for (int k = (int)(threadIdx.x & 63); k < cnt; k += 64) s += p[k];
  return warp_sum(s);
}

// Deterministic block reduction of one double per thread (blockDim.x <= 1024,
// multiple of 64). Result valid in thread 0.
__device__ inline double block_sum_double(double v, double* smem) {
  v = warp_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) smem[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) s += smem[w];
  return s;
}

// Kernel scaling: exp(-d^2 / (2 l^2)) = exp2(-d^2 * kscale2), kscale2 = log2(e)/(2 l^2).
inline double kernel_scale2(double lengthscale) { return 1.4426950408889634 / (2.0 * lengthscale * lengthscale); }

}  // namespace gpl
