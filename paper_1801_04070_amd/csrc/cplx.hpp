// Complex FP64/FP32 helpers for device code (values stored as double2 / float2 = (re, im)).
#pragma once

#include <hip/hip_runtime.h>

namespace gq {

// The fused multiply-adds are spelled out, so every kernel rounds a product the same way whatever
// the compiler would contract in its context (results of different kernels stay comparable bit
// for bit).
__host__ __device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
// |z|^2
__host__ __device__ __forceinline__ double cnorm2(double2 z) { return fma(z.x, z.x, z.y * z.y); }
__host__ __device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__host__ __device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__host__ __device__ __forceinline__ double2 cscale(double2 a, double s) {
  return make_double2(a.x * s, a.y * s);
}
// a + s * b with real s
__host__ __device__ __forceinline__ double2 caxpy(double s, double2 b, double2 a) {
  return make_double2(fma(s, b.x, a.x), fma(s, b.y, a.y));
}
// a + b * c (complex)
__host__ __device__ __forceinline__ double2 cfma(double2 b, double2 c, double2 a) {
  return make_double2(fma(b.x, c.x, fma(-b.y, c.y, a.x)), fma(b.x, c.y, fma(b.y, c.x, a.y)));
}
// 1/x for finite non-zero x: the hardware reciprocal estimate refined by two Newton steps
// (each doubles the correct bits), so the result is within an ulp or so of the division.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}

__host__ __device__ __forceinline__ double2 cinv(double2 a) {
  double s = 1.0 / cnorm2(a);
  return make_double2(a.x * s, -a.y * s);
}
// z^n for n >= 0 by binary powering
__host__ __device__ __forceinline__ double2 cpowi(double2 z, int n) {
  double2 r = make_double2(1.0, 0.0);
  while (n > 0) {
    if (n & 1) r = cmul(r, z);
    z = cmul(z, z);
    n >>= 1;
  }
  return r;
}

// FP32 overloads, used by the box-expansion kernels of the mixed-precision path.
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__host__ __device__ __forceinline__ float2 caxpy(float s, float2 b, float2 a) {
  return make_float2(fmaf(s, b.x, a.x), fmaf(s, b.y, a.y));
}
__host__ __device__ __forceinline__ float2 cfma(float2 b, float2 c, float2 a) {
  return make_float2(fmaf(b.x, c.x, fmaf(-b.y, c.y, a.x)), fmaf(b.x, c.y, fmaf(b.y, c.x, a.y)));
}

// Storage conversions between FP64 arithmetic and the expansion storage type.
__host__ __device__ __forceinline__ double2 to_d2(double2 a) { return a; }
__host__ __device__ __forceinline__ double2 to_d2(float2 a) { return make_double2(a.x, a.y); }
template <typename V> __host__ __device__ __forceinline__ V from_d2(double2 a);
template <> __host__ __device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }
template <> __host__ __device__ __forceinline__ float2 from_d2<float2>(double2 a) {
  return make_float2((float)a.x, (float)a.y);
}
template <typename V> struct Scalar;
template <> struct Scalar<double2> { using T = double; };
template <> struct Scalar<float2> { using T = float; };
template <typename V> __host__ __device__ __forceinline__ V mk2(double x, double y);
template <> __host__ __device__ __forceinline__ double2 mk2<double2>(double x, double y) {
  return make_double2(x, y);
}
template <> __host__ __device__ __forceinline__ float2 mk2<float2>(double x, double y) {
  return make_float2((float)x, (float)y);
}

}  // namespace gq
