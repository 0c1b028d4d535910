// Link-phase arithmetic shared by the U(1) and SU(2) x U(1) passes: the
// arctangent of the Cayley drift and (sin, cos - 1) of link and plaquette
// phases, with FP32 forms that need no division, no branch on the data in
// practice and no large-argument reduction.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace cl {

__device__ __forceinline__ float sin_t(float x) { return sinf(x); }
__device__ __forceinline__ double sin_t(double x) { return sin(x); }
__device__ __forceinline__ double atan_t(double x) { return atan(x); }
// FP32 arctangent: the Taylor series to u^7 where |u| <= 1/8 (truncation
// below u^9/9, i.e. 7e-9 relative), atanf elsewhere.  The link drift's
// argument e h dx pi_A / (2 a^{1-alpha}) is of order 1e-3 in practice.
__device__ __forceinline__ float atan_t(float u) {
  if (!(fabsf(u) <= 0.125f)) return atanf(u);
  const float u2 = u * u;
  return fmaf(u * u2, fmaf(u2, fmaf(u2, -1.f / 7.f, 1.f / 5.f), -1.f / 3.f), u);
}
// a / b; FP32 through the hardware reciprocal (1 ulp), which is below the
// rounding already in a and b
__device__ __forceinline__ float quot_t(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double quot_t(double a, double b) { return a / b; }

// cos t - 1 from (cos t, sin t) without cancellation: -sin^2/(1 + cos) where
// cos > 0, the plain difference (no cancellation) elsewhere
template <typename T>
__device__ __forceinline__ T cos_m1(T cs, T sn) {
  return cs > T(0) ? -quot_t(sn * sn, T(1) + cs) : cs - T(1);
}

// sin x and cos x - 1.  FP32, |x| <= 64: Cody and Waite's reduction by the
// nearest multiple k pi/2, with pi/2 split into three FP32 parts (the float
// nearest pi/2 and the two following remainders) so that r = x - k pi/2
// carries FP32 rounding only; then the Taylor series of sin r (to r^9) and of
// cos r - 1 (to r^10) on [-pi/4, pi/4], truncated below 2e-9, and the signs
// of quadrant k mod 4.  cos x - 1 comes out without cancellation for small x,
// with no division and no branch.  Other arguments and FP64 take the library
// sincos.
__device__ __forceinline__ void sincos_m1(double x, double* s, double* cm1) {
  double c;
  sincos(x, s, &c);
  *cm1 = cos_m1(c, *s);
}
__device__ __forceinline__ void sincos_m1(float x, float* s, float* cm1) {
  if (!(fabsf(x) <= 64.f)) {
    float c;
    sincosf(x, s, &c);
    *cm1 = cos_m1(c, *s);
    return;
  }
  const float k = rintf(x * 0.636619772f);
  float r = fmaf(-k, 1.57079637f, x);
  r = fmaf(-k, -4.37113883e-08f, r);
  r = fmaf(-k, -1.71512451e-15f, r);
  const float r2 = r * r;
  const float sr =
      fmaf(r * r2, fmaf(r2, fmaf(r2, fmaf(r2, 1.f / 362880.f, -1.f / 5040.f), 1.f / 120.f), -1.f / 6.f), r);
  const float cr =
      r2 * fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -1.f / 3628800.f, 1.f / 40320.f), -1.f / 720.f), 1.f / 24.f), -0.5f);
  const int q = (int)k & 3;
  // x = k pi/2 + r: (sin x, cos x) = (sin r, cos r), (cos r, -sin r),
  // (-sin r, -cos r), (-cos r, sin r) for q = 0, 1, 2, 3
  const float c1 = 1.f + cr;
  const float sb = (q & 1) ? c1 : sr, cb = (q & 1) ? sr : c1;
  *s = (q & 2) ? -sb : sb;
  const float cx = ((q + 1) & 2) ? -cb : cb;
  *cm1 = q == 0 ? cr : cx - 1.f;
}

}  // namespace cl
