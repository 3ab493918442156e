// Row generators shared by the offline and online kernels: the coefficient
// modes of the diffusion families and an FP64 exponential.
#pragma once

#include <hip/hip_runtime.h>

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

// Table-driven FP64 exponential (Tang's method): exp(t) = 2^k 2^(j/64) 2^(f/64),
// with 64 t log2(e) = 64 k + j + f, |f| <= 1/2, and 2^(f/64) from its Taylor
// series to degree 4 (truncation error < 4e-14 relative).  tab[j] = 2^(j/64)
// must be visible to the calling lanes (LDS or constant memory).
//
// exp_tab_v takes v = 64 t log2(e) directly (callers fold the factor into a
// per-parameter constant).  Only full-rate operations are used: the nearest
// integer comes from adding and subtracting 1.5 * 2^52 (round to nearest
// even in the add) and its two's-complement value is the low word of the
// sum; 2^k is applied by adding k to the exponent field of the (normal)
// product tab[j] * poly in [1, 2).  v is clamped at -64 * 1020, so results
// below 2^-1020 (far below any term the solves keep) stay normal instead of
// flushing to zero.
__device__ __forceinline__ double exp_tab_v(double v, const double* tab) {
  constexpr double c1 = 0.010830424696249145;                // ln2 / 64
  constexpr double c2 = c1 * c1 / 2.0;
  constexpr double c3 = c2 * c1 / 3.0;
  constexpr double c4 = c3 * c1 / 4.0;
  constexpr double kShift = 6755399441055744.0;               // 1.5 * 2^52
  v = fmax(v, -65280.0);
  const double sh = v + kShift;
  const double nr = sh - kShift;
  const double f = v - nr;
  const int ni = static_cast<int>(__double2loint(sh));
  const double poly = fma(fma(fma(fma(c4, f, c3), f, c2), f, c1), f, 1.0);
  const double e = tab[ni & 63] * poly;
  return __hiloint2double(__double2hiint(e) + ((ni >> 6) << 20), __double2loint(e));
}

__device__ __forceinline__ double exp_tab(double t, const double* tab) {
  constexpr double k64log2e = 92.332482616893656877;        // 64 / ln 2
  return exp_tab_v(t * k64log2e, tab);
}

}  // namespace subap
