// Per-pair FP64 arithmetic of the ULA closed forms beyond eq. (6): the uniform
// stationary-phase form of the discrete sum and the aperture quadrature for
// pairs without a stationary-phase regime.  Shared by k_closedform and the
// learned correction's pair inputs.
//
// For users i, j (perpendicular distances xi, xj, positions yi, yj along the
// array) the entry is S = sum_n f(y_n) e^{j phi(y_n)}, f = |h_i| |h_j|,
// phi = k (r_i - r_j), elements y_n = (n - (N-1)/2) d.
//
// Numeric pairs (numeric_route below: slow-phase pairs, for which k |u_i - u_j|
// times the angular span of the aperture seen from the pair's midpoint is at most
// kQuadRadPerPanel * kQuadMaxPanels, and affordable pairs with a broad stationary zone):
//   S = (1/d) int_{-L}^{L} f e^{j phi} dy  + discrete end corrections,
//   the integral by composite 64-node Gauss-Legendre in the angle theta seen
//   from the midpoint (y = y_m + x_m tan theta), one panel per kQuadRadPerPanel
//   radians of phase (|d phi / d theta| <= k |u_i - u_j|); or the direct sum
//   over the N elements when N <= kDirectMaxN or it costs no more.
// Other pairs: the uniform expansion about the stationary point y* (the
// change of variable phi - phi* = sigma s^2 / 2, sigma = sgn phi''(y*)):
//   (1/d) sum over the ends e = L (+), -L (-) of
//      +- [ G0 e^{j phi*} F(s_e) + e^{j phi(e)} (f(e) / (j phi'(e)) - G0 / (j sigma s_e)) ]
//   + discrete end corrections,
//   G0 = f(y*) / sqrt|phi''(y*)|, F(s) = int_0^s e^{j sigma t^2/2} dt.
//   |s_e| <= 8: F by kFresnelNodes-node Gauss-Legendre on [0, s_e] (at most 32 rad
//   of phase: 32 nodes reach FP64 rounding); |s_e| > 8: F's
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
constexpr double kQuadRadPerPanel = 120.0;   // phase change over one 64-node panel
constexpr int kQuadMaxPanels = 8;            // slow-phase pairs: at most 960 rad over the aperture
constexpr double kSGuard = 1e-2;
constexpr double kFresnelSplit = 8.0;
constexpr int kDirectMaxN = 1024;   // numeric pairs of arrays up to this size take the direct sum

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

// r = sqrt(r2) and 1/r without a division: the reciprocal square root from the
// FP32 estimate and one Newton step (relative error below 4e-14), then one
// correction of r = r2 / sqrt(r2), which squares that error away: r to FP64
// rounding (it feeds the phase), 1/r to 4e-14 (it feeds amplitudes only).
__device__ __forceinline__ void dist_inv(double r2, double& r, double& inv) {
  inv = rsqrt_nr1(r2);
  r = r2 * inv;
  r = fma(0.5 * inv, fma(-r, r, r2), r);
}

// 1/c for c > 0 well inside the FP32 range: the FP32 estimate and two Newton steps.
__device__ __forceinline__ double recip_nr2(double c) {
  double y = (double)__builtin_amdgcn_rcpf((float)c);
  y = fma(y, fma(-c, y, 1.0), y);
  return fma(y, fma(-c, y, 1.0), y);
}

// f(y) e^{j phi(y)} for the numeric routes (no division: amplitudes from the
// reciprocal distances); sq_ij = sqrt(x_i x_j) for PNUSW.
__device__ __forceinline__ Cplx node_val(const PairGeom& g, double y, double sq_ij) {
  const double di = y - g.yi, dj = y - g.yj;
  double ri, rj, ii, ij;
  dist_inv(fma(di, di, g.xi * g.xi), ri, ii);
  dist_inv(fma(dj, dj, g.xj * g.xj), rj, ij);
  const double u = ii * ij;
  const double amp = g.amp == XLMIMO_AMP_PNUSW ? g.beta0 * sq_ij * u * sqrt(u) : g.c_fs * u;
  return cscale(phasor_turns_d((ri - rj) * g.inv_lambda), amp);
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

// The Fresnel integrals F(s_e), |s_e| <= kFresnelSplit, that uniform_pair leaves to its
// caller: the entry still takes coef[e] F(s_e) for each end e with need[e] set.  A few
// pairs of a wave need one (about one end in twenty on the sweep's drops), so evaluating
// them in place would hold every lane of the wave for the whole node loop.
struct FresnelReq {
  bool need[2];
  double s[2], sigma[2];
  Cplx coef[2];
};

// Uniform stationary-phase entry of a fast-phase pair (see the file notes), less the
// Fresnel integrals recorded in fr (fresnel_complete adds them).
__device__ Cplx uniform_pair(const PairGeom& g, int n, double d, FresnelReq& fr) {
  const double L = 0.5 * (double)n * d;
  Cplx integral = {0.0, 0.0};
  fr.need[0] = fr.need[1] = false;
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
        // G0 e^{j phi*} F(s), scaled as the integral below: left to the caller
        fr.need[e] = true;
        fr.s[e] = s;
        fr.sigma[e] = sigma;
        fr.coef[e] = cscale(eph, se * g0 / d);
        part = {0.0, 0.0};
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

// Completes the Fresnel integrals F(s) = int_0^s e^{j sigma t^2 / 2} dt that uniform_pair
// recorded in the wave's lanes (Gauss-Legendre with kFresnelNodes = 32 nodes on [0, s]): the
// requests go two at a time to the wave's halves, lane q of a half taking node q; the nodes'
// terms are summed across the half (butterfly) and the requesting lane adds coef F to v.
// Every lane of the wave calls it (the loop trip count is the wave's, from a ballot).
// gl_f: the 32-node rule ((node, weight) pairs).
__device__ void fresnel_complete(const FresnelReq& fr, Cplx& v, const double* __restrict__ gl_f) {
  static_assert(kFresnelNodes == 32, "one node per lane of a half-wave");
  const int lane = threadIdx.x & 63, q = lane & 31, upper = lane >> 5;
  const double xq = gl_f[2 * q], wq = gl_f[2 * q + 1];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    unsigned long long pending = __ballot(fr.need[e]);
    while (pending != 0) {
      const int a = __ffsll((long long)pending) - 1;
      pending &= pending - 1;
      const int b = pending != 0 ? __ffsll((long long)pending) - 1 : -1;
      if (b >= 0) pending &= pending - 1;
      const int src = upper ? b : a;
      const double s = __shfl(fr.s[e], src < 0 ? a : src);
      const double sigma = __shfl(fr.sigma[e], src < 0 ? a : src);
      Cplx term = {0.0, 0.0};
      if (src >= 0) {
        const double t = 0.5 * s * (1.0 + xq);
        // e^{j sigma t^2/2}: t^2 / (4 pi) turns
        term = cscale(phasor_turns_d(sigma * t * t / (4.0 * kPiPair)), wq);
      }
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) {
        term.re += __shfl_xor(term.re, o);
        term.im += __shfl_xor(term.im, o);
      }
      const Cplx sa = {__shfl(term.re, 0), __shfl(term.im, 0)};
      const Cplx sb = {__shfl(term.re, 32), __shfl(term.im, 32)};
      if (lane == a || lane == b) {
        const Cplx F = cscale(lane == a ? sa : sb, 0.5 * fr.s[e]);
        v = cadd(v, cmul(fr.coef[e], F));
      }
    }
  }
}

// ---- numeric routes -----------------------------------------------------------
// Pairs evaluated numerically by the closed forms UNIFORM and GATED_QUAD: slow-phase
// pairs (<= kQuadMaxPanels panels) and pairs whose stationary zone is broad
// (Fresnel width sqrt(2 pi / |phi''(y*)|) >= L / kBroadFraction, or x_i == x_j) when
// the quadrature costs at most N / 8 nodes; the direct sum over the N elements
// replaces the quadrature for N <= kDirectMaxN or when it costs no more.
constexpr double kBroadFraction = 2.0;
enum { ROUTE_NONE = 0, ROUTE_DIRECT = 1, ROUTE_QUAD = 2 };

__device__ __forceinline__ int quad_panels(const PairGeom& g, int n, double d) {
  const double L = 0.5 * (double)n * d;
  const double xm = 0.5 * (g.xi + g.xj), ym = 0.5 * (g.yi + g.yj);
  const double span = atan((L - ym) / xm) - atan((-L - ym) / xm);
  const double dx = g.xi - g.xj, dy = g.yi - g.yj;
  const double v = g.k * sqrt(dx * dx + dy * dy) * span;
  const double p = ceil(v / kQuadRadPerPanel);
  return p < 1.0 ? 1 : (p > 1e9 ? 1000000000 : (int)p);
}

__device__ __forceinline__ int numeric_route(const PairGeom& g, int n, double d, int n_gl, int& panels) {
  const int p = quad_panels(g, n, d);
  const double L = 0.5 * (double)n * d;
  bool broad = true;
  if (g.xi != g.xj) {
    const double ys = (g.yi * g.xj - g.xi * g.yj) / (g.xj - g.xi);
    const double a = sqrt(fma(ys - g.yi, ys - g.yi, g.xi * g.xi)), b = sqrt(fma(ys - g.yj, ys - g.yj, g.xj * g.xj));
    const double p2 = g.k * (g.xi * g.xi / (a * a * a) - g.xj * g.xj / (b * b * b));
    const double lb = L / kBroadFraction;
    broad = p2 == 0.0 || 2.0 * kPiPair / fabs(p2) >= lb * lb;
  }
  panels = 0;
  if (p <= kQuadMaxPanels || (broad && (double)p * n_gl * 8.0 <= (double)n)) {
    panels = p;
    return (n <= kDirectMaxN || n <= (int64_t)p * n_gl) ? ROUTE_DIRECT : ROUTE_QUAD;
  }
  return ROUTE_NONE;
}

// This thread's share of a numeric entry when `nthr` threads (a multiple of n_gl = 64) stride
// the terms: elements t, t + nthr, ... of the direct sum, or the quadrature nodes q = t % 64 of
// panels p = t / 64, t / 64 + nthr / 64, ... (angle theta seen from the midpoint; weights and
// Jacobian included, without the 1/d).  A thread keeps one node q, so sin / cos of its offset
// within a panel are taken once and the panel midpoints advance by rotation (re-taken exactly
// every 16 steps).
__device__ Cplx numeric_share(const PairGeom& g, int n, double d, int route, int panels,
                              const double* __restrict__ gl, int n_gl, int t, int nthr) {
  Cplx acc = {0.0, 0.0};
  const double sq_ij = sqrt(g.xi * g.xj);
  if (route == ROUTE_DIRECT) {
    for (int m = t; m < n; m += nthr) acc = cadd(acc, node_val(g, ((double)m - 0.5 * (double)(n - 1)) * d, sq_ij));
    return acc;
  }
  const double L = 0.5 * (double)n * d;
  const double xm = 0.5 * (g.xi + g.xj), ym = 0.5 * (g.yi + g.yj);
  const double ta = atan((-L - ym) / xm), tb = atan((L - ym) / xm);
  const double h = (tb - ta) / panels;
  const int q = t % n_gl, pstep = nthr / n_gl;
  double sd, cd;
  sincos(0.5 * h * gl[2 * q], &sd, &cd);
  const double wq = 0.5 * h * gl[2 * q + 1] * xm;
  double ss, cs;
  sincos(pstep * h, &ss, &cs);
  double sm = 0.0, cm = 1.0;
  int it = 0;
  for (int p = t / n_gl; p < panels; p += pstep, ++it) {
    if ((it & 15) == 0) {
      sincos(ta + (p + 0.5) * h, &sm, &cm);
    }
    const double c = cm * cd - sm * sd, s = sm * cd + cm * sd;  // cos, sin of the node angle
    const double ic = recip_nr2(c);
    const double y = fma(xm * s, ic, ym);
    acc = cadd(acc, cscale(node_val(g, y, sq_ij), wq * ic * ic));
    const double sn = sm * cs + cm * ss;
    cm = cm * cs - sm * ss;
    sm = sn;
  }
  return acc;
}

// Fixed-order sum over the 64 lanes of a wave (butterfly; every lane ends with the same value).
__device__ __forceinline__ Cplx wave_sum_c(Cplx v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_xor(v.re, o, 64);
    v.im += __shfl_xor(v.im, o, 64);
  }
  return v;
}

}  // namespace xl
