// Device arithmetic for on-the-fly spherical-wave channel entries (gfx950).
//
// A channel entry (eq. (3), or the free-space model) needs the element-user
// distance r, the phase 2 pi r / lambda and an amplitude.  Phases reach 1e5
// revolutions, so r and r / lambda stay in FP64 and only the reduced phase
// (|t| <= 1/8 revolution after removing whole quarter turns) goes to FP32 for
// the sin/cos of the FP32C path.
//
//  * rsqrt_nr1/rsqrt_nr2: 1/sqrt(r^2) from the hardware FP32 estimate
//    (v_rsq_f32, ~1 ulp) refined by one or two Newton steps in FP64:
//    relative error ~1.5 eps32^2 = 2e-14 after one step, FP64 rounding after two.
//  * reduce_quarter: u = m + q/4 + t with integer m, q in 0..3, |t| <= 1/8.
//  * sincos_rev: sin(2 pi t), cos(2 pi t) for |t| <= 1/8 by Taylor series in t
//    (coefficients (2 pi)^n / n! evaluated at compile time).  Truncation
//    error: FP32 (sin to t^9, cos to t^10) < 2e-9; FP64 (sin to t^17, cos to
//    t^18) < 1e-19.
//  * sincos_quarter: sin(pi t / 2), cos(pi t / 2) for |t| <= 1/2 (the same
//    angles, with t in quarter turns), coefficients (pi/2)^n / n!.
//  * sincos_half: sin(pi t), cos(pi t) for |t| <= 1/2 (t in half turns),
//    coefficients pi^n / n!.  Truncation error: FP32 (sin to t^13, cos to t^12)
//    < 7e-9; FP64 (sin to t^21, cos to t^22) < 1e-17.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xl {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr double kTwoPi = 6.28318530717958647692528676655900577;

constexpr double kHalfPi = 1.57079632679489661923132169163975144;

constexpr double taylor_coef_w(int n, double w) {
  // w^n / n! with the alternating sign of the sin (odd n) / cos (even n) series
  double v = 1.0;
  for (int i = 1; i <= n; ++i) v *= w / i;
  const int k = n / 2;
  return (k % 2) ? -v : v;
}
constexpr double taylor_coef(int n) { return taylor_coef_w(n, kTwoPi); }
constexpr double quarter_coef(int n) { return taylor_coef_w(n, kHalfPi); }
constexpr double half_coef(int n) { return taylor_coef_w(n, 2.0 * kHalfPi); }

// a * b + c in FP64 with the coefficient c in scalar registers.  The Horner steps of the
// series below otherwise become the two-operand v_fmac_f64, which needs the addend in the
// destination: with the coefficients held in vector registers across a loop, every step
// then costs a 64-bit copy on top of the multiply-add.
__device__ __forceinline__ double fma_sc(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}
// A Horner step with the coefficient in scalar registers (SC) or placed by the compiler.  The
// scalar form pays off where waves have registers to spare; in a kernel that runs one wave per
// SIMD with every vector register taken, the plain form was the faster one (the FP64 exact Gram
// of three- and four-block items: 162 against 181 ms for twenty 1000-user drops).
template <bool SC>
__device__ __forceinline__ double horner_step(double a, double b, double c) {
  if constexpr (SC) return fma_sc(a, b, c);
  return fma(a, b, c);
}

__device__ __forceinline__ double rsqrt_nr1(double r2) {
  double y = (double)__builtin_amdgcn_rsqf((float)r2);
  double e = fma(-r2 * y, y, 1.0);  // 1 - r2 y^2
  return fma(0.5 * y, e, y);
}

__device__ __forceinline__ double rsqrt_nr2(double r2) {
  double y = rsqrt_nr1(r2);
  double e = fma(-r2 * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// u >= 0 in revolutions -> (t, q): u = integer + q / 4 + t
__device__ __forceinline__ void reduce_quarter(double u, double& t, int& q) {
  double q4 = __builtin_rint(4.0 * u);
  t = fma(q4, -0.25, u);
  q = ((int)q4) & 3;
}

__device__ __forceinline__ void sincos_rev(float t, float& s, float& c) {
  const float t2 = t * t;
  float ps = (float)taylor_coef(9);
  ps = fmaf(ps, t2, (float)taylor_coef(7));
  ps = fmaf(ps, t2, (float)taylor_coef(5));
  ps = fmaf(ps, t2, (float)taylor_coef(3));
  ps = fmaf(ps, t2, (float)taylor_coef(1));
  s = ps * t;
  float pc = (float)taylor_coef(10);
  pc = fmaf(pc, t2, (float)taylor_coef(8));
  pc = fmaf(pc, t2, (float)taylor_coef(6));
  pc = fmaf(pc, t2, (float)taylor_coef(4));
  pc = fmaf(pc, t2, (float)taylor_coef(2));
  c = fmaf(pc, t2, 1.0f);
}

__device__ __forceinline__ void sincos_rev(double t, double& s, double& c) {
  const double t2 = t * t;
  double ps = taylor_coef(17);
#pragma unroll
  for (int n = 15; n >= 1; n -= 2) ps = fma_sc(ps, t2, taylor_coef(n));
  s = ps * t;
  double pc = taylor_coef(18);
#pragma unroll
  for (int n = 16; n >= 2; n -= 2) pc = fma_sc(pc, t2, taylor_coef(n));
  c = fma(pc, t2, 1.0);
}

__device__ __forceinline__ void sincos_quarter(float t, float& s, float& c) {
  const float t2 = t * t;
  float ps = (float)quarter_coef(9);
  ps = fmaf(ps, t2, (float)quarter_coef(7));
  ps = fmaf(ps, t2, (float)quarter_coef(5));
  ps = fmaf(ps, t2, (float)quarter_coef(3));
  ps = fmaf(ps, t2, (float)quarter_coef(1));
  s = ps * t;
  float pc = (float)quarter_coef(10);
  pc = fmaf(pc, t2, (float)quarter_coef(8));
  pc = fmaf(pc, t2, (float)quarter_coef(6));
  pc = fmaf(pc, t2, (float)quarter_coef(4));
  pc = fmaf(pc, t2, (float)quarter_coef(2));
  c = fmaf(pc, t2, 1.0f);
}

__device__ __forceinline__ void sincos_quarter(double t, double& s, double& c) {
  const double t2 = t * t;
  double ps = quarter_coef(17);
#pragma unroll
  for (int n = 15; n >= 1; n -= 2) ps = fma_sc(ps, t2, quarter_coef(n));
  s = ps * t;
  double pc = quarter_coef(18);
#pragma unroll
  for (int n = 16; n >= 2; n -= 2) pc = fma_sc(pc, t2, quarter_coef(n));
  c = fma(pc, t2, 1.0);
}

// sin(pi t), cos(pi t), |t| <= 1/2; `neg_sin` returns -sin(pi t) (sign folded into the coefficients).
__device__ __forceinline__ void sincos_half(float t, float& ns, float& c) {
  const float t2 = t * t;
  float ps = (float)-half_coef(13);
#pragma unroll
  for (int n = 11; n >= 1; n -= 2) ps = fmaf(ps, t2, (float)-half_coef(n));
  ns = ps * t;
  float pc = (float)half_coef(12);
#pragma unroll
  for (int n = 10; n >= 2; n -= 2) pc = fmaf(pc, t2, (float)half_coef(n));
  c = fmaf(pc, t2, 1.0f);
}

template <bool SC = true>
__device__ __forceinline__ void sincos_half(double t, double& ns, double& c) {
  const double t2 = t * t;
  double ps = -half_coef(21);
#pragma unroll
  for (int n = 19; n >= 1; n -= 2) ps = horner_step<SC>(ps, t2, -half_coef(n));
  ns = ps * t;
  double pc = half_coef(22);
#pragma unroll
  for (int n = 20; n >= 2; n -= 2) pc = horner_step<SC>(pc, t2, half_coef(n));
  c = fma(pc, t2, 1.0);
}

// a * exp(-j 2 pi (q/4 + t)) given s = sin(2 pi t), c = cos(2 pi t).
// exp(-j phi) = (cos phi, -sin phi); a quarter turn q rotates (c, s).
template <typename T>
__device__ __forceinline__ void rotate_conj(T a, T s, T c, int q, T& re, T& im) {
  const bool swap = q & 1;
  const T x = swap ? s : c;
  const T y = swap ? c : s;
  const T ar = (q == 1 || q == 2) ? -a : a;
  const T ai = (q < 2) ? -a : a;
  re = x * ar;
  im = y * ai;
}

}  // namespace xl
