// Forward-mode dual numbers with D tangent directions (FP32), used to obtain
// per-point Jacobians of the ray tracer by running the same templated code.
#pragma once

#include <hip/hip_runtime.h>

namespace gpl {

template <int D>
struct Dual {
  float v;
  float d[D];
  __device__ Dual() : v(0.f) {
#pragma unroll
    for (int k = 0; k < D; ++k) d[k] = 0.f;
  }
  __device__ Dual(float x) : v(x) {
#pragma unroll
    for (int k = 0; k < D; ++k) d[k] = 0.f;
  }
  __device__ static Dual var(float x, int dir) {
    Dual r(x);
    r.d[dir] = 1.f;
    return r;
  }
};

#define GPL_DUAL_BIN(OP, VAL, DER)                                           \
  template <int D>                                                           \
  __device__ inline Dual<D> operator OP(const Dual<D>& a, const Dual<D>& b) { \
    Dual<D> r;                                                               \
    r.v = VAL;                                                               \
    _Pragma("unroll") for (int k = 0; k < D; ++k) r.d[k] = DER;              \
    return r;                                                                \
  }
GPL_DUAL_BIN(+, a.v + b.v, a.d[k] + b.d[k])
GPL_DUAL_BIN(-, a.v - b.v, a.d[k] - b.d[k])
GPL_DUAL_BIN(*, a.v * b.v, a.d[k] * b.v + a.v * b.d[k])
#undef GPL_DUAL_BIN

template <int D>
__device__ inline Dual<D> operator/(const Dual<D>& a, const Dual<D>& b) {
  Dual<D> r;
  const float inv = 1.f / b.v;
  r.v = a.v * inv;
#pragma unroll
  for (int k = 0; k < D; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * inv;
  return r;
}
template <int D>
__device__ inline Dual<D> operator-(const Dual<D>& a) {
  Dual<D> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < D; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int D>
__device__ inline Dual<D> operator+(const Dual<D>& a, float b) { Dual<D> r = a; r.v += b; return r; }
template <int D>
__device__ inline Dual<D> operator+(float b, const Dual<D>& a) { Dual<D> r = a; r.v += b; return r; }
template <int D>
__device__ inline Dual<D> operator-(const Dual<D>& a, float b) { Dual<D> r = a; r.v -= b; return r; }
template <int D>
__device__ inline Dual<D> operator-(float b, const Dual<D>& a) { return -(a - b); }
template <int D>
__device__ inline Dual<D> operator*(const Dual<D>& a, float b) {
  Dual<D> r;
  r.v = a.v * b;
#pragma unroll
  for (int k = 0; k < D; ++k) r.d[k] = a.d[k] * b;
  return r;
}
template <int D>
__device__ inline Dual<D> operator*(float b, const Dual<D>& a) { return a * b; }

template <int D>
__device__ inline Dual<D> dsqrt(const Dual<D>& a) {
  Dual<D> r;
  r.v = sqrtf(a.v);
  const float h = 0.5f / r.v;
#pragma unroll
  for (int k = 0; k < D; ++k) r.d[k] = a.d[k] * h;
  return r;
}
template <int D>
__device__ inline Dual<D> dexp2(const Dual<D>& a) {
  Dual<D> r;
  r.v = exp2f(a.v);
  const float h = r.v * 0.69314718055994531f;
#pragma unroll
  for (int k = 0; k < D; ++k) r.d[k] = a.d[k] * h;
  return r;
}
template <int D>
__device__ inline Dual<D> dlog2(const Dual<D>& a) {
  Dual<D> r;
  r.v = log2f(a.v);
  const float h = 1.4426950408889634f / a.v;
#pragma unroll
  for (int k = 0; k < D; ++k) r.d[k] = a.d[k] * h;
  return r;
}
template <int D>
__device__ inline Dual<D> dcos(const Dual<D>& a) {
  Dual<D> r;
  float s, c;
  sincosf(a.v, &s, &c);
  r.v = c;
#pragma unroll
  for (int k = 0; k < D; ++k) r.d[k] = -s * a.d[k];
  return r;
}
template <int D>
__device__ inline Dual<D> dsin(const Dual<D>& a) {
  Dual<D> r;
  float s, c;
  sincosf(a.v, &s, &c);
  r.v = s;
#pragma unroll
  for (int k = 0; k < D; ++k) r.d[k] = c * a.d[k];
  return r;
}

// Plain-float overloads so templated code reads the same for both types.
__device__ inline float dsqrt(float a) { return sqrtf(a); }
__device__ inline float dexp2(float a) { return exp2f(a); }
__device__ inline float dlog2(float a) { return log2f(a); }
__device__ inline float dcos(float a) { return cosf(a); }
__device__ inline float dsin(float a) { return sinf(a); }
__device__ inline float value_of(float a) { return a; }
template <int D>
__device__ inline float value_of(const Dual<D>& a) { return a.v; }

}  // namespace gpl
