// Per-pair FP64 arithmetic of the ULA closed forms beyond eq. (6): the uniform
// stationary-phase form of the discrete sum and the aperture quadrature for
// pairs without a stationary-phase regime.  Shared by k_closedform and the
// learned correction's pair inputs.
//
// For users i, j (perpendicular distances xi, xj, positions yi, yj along the
// array) the entry is S = sum_n f(y_n) e^{j phi(y_n)}, f = |h_i| |h_j|,
// phi = k (r_i - r_j), elements y_n = (n - (N-1)/2) d.
//
// Slow-phase pairs (k |u_i - u_j| times the angular span of the aperture seen
// from the pair's midpoint <= kQuadRadPerPanel * kQuadMaxPanels):
//   S = (1/d) int_{-L}^{L} f e^{j phi} dy  + discrete end corrections,
//   the integral by composite 64-node Gauss-Legendre in the angle theta seen
//   from the midpoint (y = y_m + x_m tan theta), one panel per kQuadRadPerPanel
//   radians of phase (|d phi / d theta| <= k |u_i - u_j|).
// Fast-phase pairs: the uniform expansion about the stationary point y* (the
// change of variable phi - phi* = sigma s^2 / 2, sigma = sgn phi''(y*)):
//   (1/d) sum over the ends e = L (+), -L (-) of
//      +- [ G0 e^{j phi*} F(s_e) + e^{j phi(e)} (f(e) / (j phi'(e)) - G0 / (j sigma s_e)) ]
//   + discrete end corrections,
//   G0 = f(y*) / sqrt|phi''(y*)|, F(s) = int_0^s e^{j sigma t^2/2} dt.
//   |s_e| <= 8: F by 64-node Gauss-Legendre on [0, s_e]; |s_e| > 8: F's
//   asymptotic series sgn(s) sqrt(pi/2) e^{j sigma pi/4} + e^{j sigma s^2/2}
//   / (j sigma s) (1 + Q(s)), Q = sum_{m>=1} (2m-1)!! / (j sigma s^2)^m, folded into
//   the end term so that its leading part cancels analytically.
//   |s_e| < kSGuard: the end bracket (a difference of two terms that diverge as
//   y* reaches the end) is interpolated linearly between y* -+ kSGuard/sqrt|phi''|.
//   xi == xj (no stationary point): the end terms f e^{j phi} / (j phi') alone.
// Discrete end corrections (sum minus cell integral at each end element for a
// locally linear phase theta = phi'(y_e) d):
//   +- f(y_e) e^{j phi(y_e)} e^{+-j theta/2} / j [1/(2 sin(theta/2)) - 1/theta].
#pragma once

#include "device_math.h"
#include "internal.h"
#include "xlmimo.h"

namespace xl {

constexpr double kPiPair = 3.14159265358979323846264338327950288;
constexpr double kQuadRadPerPanel = 40.0;
constexpr int kQuadMaxPanels = 16;
constexpr double kSGuard = 1e-2;
constexpr double kFresnelSplit = 8.0;

struct Cplx {
  double re, im;
};

__device__ __forceinline__ Cplx cmul(Cplx a, Cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Cplx cadd(Cplx a, Cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cplx cscale(Cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ Cplx cdiv(Cplx a, Cplx b) {
  const double den = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}

// e^{j 2 pi u} for a phase u in turns (FP64, Taylor sin/cos of the half-turn remainder)
__device__ __forceinline__ Cplx phasor_turns_d(double u) {
  const double v = 2.0 * u;
  const double q = __builtin_rint(v);
  double ns, c;
  sincos_half(v - q, ns, c);
  const double sg = (((long long)q) & 1) ? -1.0 : 1.0;
  return {sg * c, -sg * ns};
}

struct PairGeom {
  double xi, yi, xj, yj;  // perpendicular distances and positions along the array
  double k;               // 2 pi / lambda
  double inv_lambda;
  int amp;
  double beta0, c_fs;     // PNUSW beta0, free-space (lambda / 4 pi)^2
};

__device__ __forceinline__ double amp_product(const PairGeom& g, double ri, double rj) {
  if (g.amp == XLMIMO_AMP_PNUSW) {
    const double p = ri * rj;
    return g.beta0 * sqrt(g.xi * g.xj) / (p * sqrt(p));
  }
  return g.c_fs / (ri * rj);
}

// f(y) e^{j phi(y)}, phi'(y), and the distances
struct EndVals {
  Cplx g;
  double dphi;
  double ri, rj;
};

__device__ __forceinline__ EndVals end_vals(const PairGeom& g, double y) {
  const double di = y - g.yi, dj = y - g.yj;
  const double ri = sqrt(fma(di, di, g.xi * g.xi)), rj = sqrt(fma(dj, dj, g.xj * g.xj));
  EndVals v;
  v.ri = ri;
  v.rj = rj;
  v.g = cscale(phasor_turns_d((ri - rj) * g.inv_lambda), amp_product(g, ri, rj));
  v.dphi = g.k * (di / ri - dj / rj);
  return v;
}

// 1 / (2 sin(t/2)) - 1/t, by its series near 0
__device__ __forceinline__ double half_cosec_minus_inverse(double t) {
  if (fabs(t) < 1e-2) {
    const double t2 = t * t;
    return t * (1.0 / 24.0 + t2 * (7.0 / 5760.0 + t2 * (31.0 / 967680.0)));
  }
  return 1.0 / (2.0 * sin(0.5 * t)) - 1.0 / t;
}

// Sum minus cell integral at both end elements (locally linear phase).
__device__ Cplx discrete_end_corrections(const PairGeom& g, int n, double d) {
  const double y_top = 0.5 * (double)(n - 1) * d;
  Cplx total = {0.0, 0.0};
  for (int e = 0; e < 2; ++e) {
    const double side = e == 0 ? 1.0 : -1.0;
    const EndVals v = end_vals(g, side * y_top);
    const double th = v.dphi * d;
    const double c = half_cosec_minus_inverse(th);
    // side * g * e^{j side th/2} / j * c
    const Cplx rot = {cos(0.5 * side * th), sin(0.5 * side * th)};
    const Cplx t = cmul(v.g, rot);
    total = cadd(total, cscale(Cplx{t.im, -t.re}, side * c));
  }
  return total;
}

// Panels of the aperture quadrature, 0 for a fast-phase pair.
__device__ __forceinline__ int slow_panels(const PairGeom& g, int n, double d) {
  const double L = 0.5 * (double)n * d;
  const double xm = 0.5 * (g.xi + g.xj), ym = 0.5 * (g.yi + g.yj);
  const double span = atan((L - ym) / xm) - atan((-L - ym) / xm);
  const double dx = g.xi - g.xj, dy = g.yi - g.yj;
  const double v = g.k * sqrt(dx * dx + dy * dy) * span;
  int p = (int)ceil(v / kQuadRadPerPanel);
  if (p < 1) p = 1;
  return p <= kQuadMaxPanels ? p : 0;
}

// (1/d) int_{-L}^{L} f e^{j phi} dy, composite Gauss-Legendre in the midpoint's angle.
__device__ Cplx aperture_quadrature(const PairGeom& g, int n, double d, int panels, const double* __restrict__ gl,
                                    int n_gl) {
  const double L = 0.5 * (double)n * d;
  const double xm = 0.5 * (g.xi + g.xj), ym = 0.5 * (g.yi + g.yj);
  const double ta = atan((-L - ym) / xm), tb = atan((L - ym) / xm);
  const double h = (tb - ta) / panels;
  Cplx total = {0.0, 0.0};
  for (int p = 0; p < panels; ++p) {
    const double mid = ta + (p + 0.5) * h, half = 0.5 * h;
    Cplx acc = {0.0, 0.0};
    for (int q = 0; q < n_gl; ++q) {
      const double th = fma(half, gl[2 * q], mid);
      double s, c;
      sincos(th, &s, &c);
      const double y = fma(xm, s / c, ym);
      const double jac = xm / (c * c);
      const EndVals v = end_vals(g, y);
      acc = cadd(acc, cscale(v.g, gl[2 * q + 1] * jac));
    }
    total = cadd(total, cscale(acc, half));
  }
  return cscale(total, 1.0 / d);
}

// F(s) = int_0^s e^{j sigma t^2 / 2} dt for |s| <= kFresnelSplit (Gauss-Legendre on [0, s]).
__device__ Cplx fresnel_small(double s, double sigma, const double* __restrict__ gl, int n_gl) {
  const double half = 0.5 * s;
  Cplx acc = {0.0, 0.0};
  for (int q = 0; q < n_gl; ++q) {
    const double t = half * (1.0 + gl[2 * q]);
    // e^{j sigma t^2/2}: t^2 / (4 pi) turns
    const Cplx e = phasor_turns_d(sigma * t * t / (4.0 * kPiPair));
    acc = cadd(acc, cscale(e, gl[2 * q + 1]));
  }
  return cscale(acc, half);
}

// Uniform stationary-phase entry of a fast-phase pair (see the file notes).
__device__ Cplx uniform_pair(const PairGeom& g, int n, double d, const double* __restrict__ gl, int n_gl) {
  const double L = 0.5 * (double)n * d;
  Cplx integral = {0.0, 0.0};
  if (g.xi == g.xj) {
    for (int e = 0; e < 2; ++e) {
      const double se = e == 0 ? 1.0 : -1.0;
      const EndVals v = end_vals(g, se * L);
      // se * g / (j phi')
      integral = cadd(integral, cscale(Cplx{v.g.im, -v.g.re}, se / v.dphi));
    }
  } else {
    const double ys = (g.yi * g.xj - g.xi * g.yj) / (g.xj - g.xi);
    const EndVals vs = end_vals(g, ys);
    const double p2 = g.k * (g.xi * g.xi / (vs.ri * vs.ri * vs.ri) - g.xj * g.xj / (vs.rj * vs.rj * vs.rj));
    const double sigma = p2 > 0.0 ? 1.0 : -1.0;
    const double sq = sqrt(fabs(p2));
    const double g0 = amp_product(g, vs.ri, vs.rj) / sq;
    const Cplx eph = phasor_turns_d((vs.ri - vs.rj) * g.inv_lambda);  // e^{j phi*}
    // s(y) from r(y) - r(y*) = (y - y*)(y + y* - 2 y_u) / (r(y) + r(y*))
    auto s_of = [&](double y, const EndVals& v) {
      const double dr = (y - ys) * ((y + ys - 2.0 * g.yi) / (v.ri + vs.ri) - (y + ys - 2.0 * g.yj) / (v.rj + vs.rj));
      return copysign(sqrt(2.0 * g.k * fabs(dr)), y - ys);
    };
    // e^{j phi(y)} (f / (j phi') - g0 / (j sigma s))
    auto bracket = [&](double y) {
      const EndVals v = end_vals(g, y);
      const double s = s_of(y, v);
      // g/(j phi') = (g.im, -g.re)/phi';  e^{j phi} g0/(j sigma s) = (e.im, -e.re) g0 sigma / s
      const double a = 1.0 / v.dphi;
      const Cplx e = cscale(v.g, 1.0 / amp_product(g, v.ri, v.rj));
      const double b = g0 * sigma / s;
      return Cplx{v.g.im * a - e.im * b, -v.g.re * a + e.re * b};
    };
    for (int e = 0; e < 2; ++e) {
      const double se = e == 0 ? 1.0 : -1.0;
      const double y = se * L;
      const EndVals v = end_vals(g, y);
      const double s = s_of(y, v);
      Cplx part;
      if (fabs(s) > kFresnelSplit) {
        // G0 e^{j phi*} sgn(s) sqrt(pi/2) e^{j sigma pi/4} + e^{j phi(e)} (f/(j phi') + G0 Q(s) / (j sigma s))
        const double r2 = sqrt(0.5 * kPiPair) * (s > 0.0 ? 1.0 : -1.0) * g0;
        const double c4 = 0.70710678118654752440084436210484903;
        part = cmul(eph, Cplx{r2 * c4, r2 * sigma * c4});
        // Q(s): terms t_m = t_{m-1} (2m-1) / (j sigma s^2), t_0 = 1
        const double is2 = 1.0 / (s * s);
        Cplx t = {1.0, 0.0}, Q = {0.0, 0.0};
        for (int m = 1; m < 64; ++m) {
          const double c = (2.0 * m - 1.0) * is2;
          // multiply by c / (j sigma) = -j sigma c
          t = Cplx{t.im * sigma * c, -t.re * sigma * c};
          if (c > 1.0) break;  // past the smallest term of the asymptotic series
          Q = cadd(Q, t);
          if (fabs(t.re) + fabs(t.im) < 1e-18) break;
        }
        const Cplx e_phi = cscale(v.g, 1.0 / amp_product(g, v.ri, v.rj));
        // f/(j phi') e^{j phi} = (g.im, -g.re)/phi'
        Cplx endt = {v.g.im / v.dphi, -v.g.re / v.dphi};
        // e^{j phi} G0 Q / (j sigma s) = e^{j phi} Q (-j sigma G0 / s)
        const Cplx qq = cmul(e_phi, Q);
        const double f = g0 * sigma / s;
        endt = cadd(endt, Cplx{qq.im * f, -qq.re * f});
        part = cadd(part, endt);
      } else {
        const Cplx F = fresnel_small(s, sigma, gl, n_gl);
        part = cmul(cscale(eph, g0), F);
        Cplx br;
        if (fabs(s) < kSGuard) {
          const double hh = kSGuard / sq;
          const Cplx bm = bracket(ys - hh), bp = bracket(ys + hh);
          const double w = (y - (ys - hh)) / (2.0 * hh);
          br = Cplx{bm.re + w * (bp.re - bm.re), bm.im + w * (bp.im - bm.im)};
        } else {
          br = bracket(y);
        }
        part = cadd(part, br);
      }
      integral = cadd(integral, cscale(part, se));
    }
  }
  return cadd(cscale(integral, 1.0 / d), discrete_end_corrections(g, n, d));
}

// Uniform closed-form entry of any pair: quadrature if slow, uniform expansion if fast.
__device__ __forceinline__ Cplx uniform_entry(const PairGeom& g, int n, double d, const double* __restrict__ gl,
                                              int n_gl) {
  const int p = slow_panels(g, n, d);
  if (p > 0) return cadd(aperture_quadrature(g, n, d, p, gl, n_gl), discrete_end_corrections(g, n, d));
  return uniform_pair(g, n, d, gl, n_gl);
}

}  // namespace xl
