// Row generators shared by the offline and online kernels: the coefficient
// modes of the diffusion families and FP64 powers of two for the Gaussian
// kernel rows.
#pragma once

#include <hip/hip_runtime.h>

#include "exp2_poly.h"

namespace subap {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Modes phi_q at a point of the unit square / cube (see subap.h).
__device__ __forceinline__ void modes2d(double x, double y, double* phi) {
  phi[0] = sin(kTwoPi * x);
  phi[1] = cos(kTwoPi * y);
}

__device__ __forceinline__ void modes3d(double x, double y, double z, double* phi) {
  const double sx = sin(kTwoPi * x), cx = cos(kTwoPi * x);
  const double sy = sin(kTwoPi * y), cy = cos(kTwoPi * y);
  const double sz = sin(kTwoPi * z), cz = cos(kTwoPi * z);
  phi[0] = sx * cy;
  phi[1] = sy * cz;
  phi[2] = sz * cx;
  phi[3] = cx * cy * cz;
}

// FP64 powers of two without tables.  2^v = 2^k 2^f with k the integer
// nearest to v and |f| <= 1/2; 2^f from the near-minimax polynomial of degree
// DEG in exp2_poly.h (relative error 5.5e-11, 1.9e-14 and 2.2e-16 for DEG = 7,
// 9, 11, Horner evaluation included) and 2^k from ldexp.  k comes from adding
// 1.5 * 2^52, which rounds to the nearest integer and leaves k in
// two's complement in the low word of the sum.

template <int DEG>
__device__ __forceinline__ double exp2_reduced(double f) {
  double p = Exp2Poly<DEG>::c[DEG];
#pragma unroll
  for (int i = DEG - 1; i >= 0; --i) p = fma(p, f, Exp2Poly<DEG>::c[i]);
  return p;
}

constexpr double kRoundShift = 6755399441055744.0;  // 1.5 * 2^52
constexpr double kExp2Range = 1073741824.0;          // 2^30

// 2^(c d).  The product is not rounded before the reduction: f = c d - k comes
// from one fused multiply-add.  Requires |c d| < 2^30 (callers check a bound
// once per block); then k fits the low word and ldexp returns 0 or inf where
// the power leaves the FP64 range.
template <int DEG>
__device__ __forceinline__ double exp2_mul(double c, double d) {
  const double sh = fma(c, d, kRoundShift);
  const double k = sh - kRoundShift;
  const double f = fma(c, d, -k);
  return ldexp(exp2_reduced<DEG>(f), static_cast<int>(__double2loint(sh)));
}

// 2^v for any v: v is clamped to [-2^30, 2^30] first, which changes no
// finite result (2^-2^30 is 0 and 2^2^30 is inf in FP64); NaN gives 0.
template <int DEG>
__device__ __forceinline__ double exp2_any(double v) {
  v = fmin(fmax(v, -kExp2Range), kExp2Range);
  const double sh = v + kRoundShift;
  const double k = sh - kRoundShift;
  return ldexp(exp2_reduced<DEG>(v - k), static_cast<int>(__double2loint(sh)));
}

}  // namespace subap
