// Closed-form Gram of the paper's modified ZF (eqs. (22)-(23)): O(K^2) per drop,
// no loop over antennas.
//
// Diagonal G~_ii (P_i / P):
//   ULA PNUSW      eq. (4) with half-aperture L = N d / 2:  beta0 / (d x) S,
//                  S = (L - y)/sqrt(x^2 + (L - y)^2) + (L + y)/sqrt(x^2 + (L + y)^2)
//   ULA FREESPACE  (lambda/4pi)^2 / (d x) [atan((L - y)/x) + atan((L + y)/x)]
//   UPA PNUSW      beta0 / d^2 * solid angle of the panel seen from the user
//   UPA FREESPACE  (lambda/4pi)^2 / d^2 * int int du dv / (x^2 + u^2 + v^2) over the
//                  panel: inner integral in closed form (atan), outer by
//                  Gauss-Legendre on each side of the user's foot point.
// Off-diagonal (stationary phase; the stationary point is where the line through
// both users meets the array):
//   ULA PNUSW      rho_ij of eq. (6) (sgn of eq. (7)) times sqrt(G~_ii G~_jj), eq. (23)
//   ULA FREESPACE  (lambda/4pi)^2 sqrt(lambda) / (d sqrt(x_i x_j d_ij)) e^{j s (k d_ij - pi/4)}
//   UPA PNUSW      beta0 lambda / (d^2 d_ij) e^{j s (k d_ij - pi/2)}
//   UPA FREESPACE  (lambda/4pi)^2 lambda / (d^2 |x_i - x_j|) e^{j s (k d_ij - pi/2)}
//   with s = sgn(|x_i| - |x_j|).  Variant GATED zeroes the entry when the
//   stationary point is off the aperture; |x_i| == |x_j| or d_ij == 0 gives 0.
// Variant GATED_QUAD (ULA): GATED, except the numerically routed pairs
//   (slow-phase pairs and broad stationary zones, pair_math.h), which take the
//   aperture quadrature or the direct sum.
// Variant UNIFORM (ULA): the uniform stationary-phase form of the discrete sum,
//   with the same numeric routes (pair_math.h).
// For UNIFORM and GATED_QUAD two kernels run: k_cf_pairs takes every pair of the
//   batch on its own thread (analytic entries, and each pair's route), then
//   k_closedform takes each drop on a workgroup (the diagonal and the numeric
//   pairs: direct sums from channels staged in LDS or one wave per pair,
//   quadratures by the whole workgroup one at a time with nodes strided over the
//   threads, fixed-order wave sums, waves summed in order).
// All arithmetic is FP64; the phase d_ij / lambda is reduced in revolutions.
#include "device_math.h"
#include "internal.h"
#include "pair_math.h"
#include "xlmimo.h"

namespace xl {

constexpr double kPi = 3.14159265358979323846264338327950288;

__device__ double upa_freespace_integral(double x, double u1, double u2, double v1, double v2,
                                         const double* __restrict__ gl, int n_gl) {
  // int_{u1}^{u2} (atan(v2/a) - atan(v1/a)) / a du,  a = sqrt(x^2 + u^2);  split at u = 0
  double total = 0.0;
  double seg[3] = {u1, u2, u2};
  int nseg = 1;
  if (u1 < 0.0 && u2 > 0.0) {
    seg[1] = 0.0;
    seg[2] = u2;
    nseg = 2;
  }
  for (int s = 0; s < nseg; ++s) {
    const double lo = seg[s], hi = seg[s + 1];
    const double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
    double acc = 0.0;
    for (int i = 0; i < n_gl; ++i) {
      const double u = fma(half, gl[2 * i], mid);
      const double a = sqrt(fma(u, u, x * x));
      acc = fma(gl[2 * i + 1], (atan(v2 / a) - atan(v1 / a)) / a, acc);
    }
    total = fma(half, acc, total);
  }
  return total;
}

__device__ double solid_angle_rect(double x, double u1, double u2, double v1, double v2) {
  auto f = [x](double u, double v) { return atan(u * v / (x * sqrt(x * x + u * u + v * v))); };
  return f(u2, v2) - f(u1, v2) - f(u2, v1) + f(u1, v1);
}

// ULA user i: perpendicular distance x, position y along the array, closed-form
// diagonal G~_ii and (PNUSW) the aperture factor S of eq. (4).  ok is false for
// a user on the array line or with non-finite coordinates.  The pair kernel needs
// the free-space diagonal only to know that it is finite: with diag_value false it
// takes diag = c_fs / (d x), finite exactly when the diagonal is (the arctangent sum
// is bounded and nonzero), and skips the two FP64 arctangents.
struct UlaUser {
  double x, y, diag, sfac;
  bool ok;
};

__device__ __forceinline__ UlaUser ula_user(const ArrayK& arr, const double* __restrict__ p, double Ly, double c_fs,
                                            bool diag_value = true) {
  UlaUser u;
  const double px = p[0], py = p[1], pz = p[2];
  u.x = sqrt(fma(px, px, pz * pz));
  u.y = py;
  u.sfac = 0.0;
  u.ok = u.x > 0.0 && isfinite(u.x) && isfinite(py) && isfinite(pz);
  const double d = arr.spacing;
  if (!u.ok) {
    u.diag = __builtin_nan("");
  } else if (arr.amp == XLMIMO_AMP_PNUSW) {
    const double a = Ly - py, b = Ly + py;
    u.sfac = a / sqrt(fma(a, a, u.x * u.x)) + b / sqrt(fma(b, b, u.x * u.x));
    u.diag = arr.beta0 / (d * u.x) * u.sfac;
  } else if (diag_value) {
    u.diag = c_fs / (d * u.x) * (atan((Ly - py) / u.x) + atan((Ly + py) / u.x));
  } else {
    u.diag = c_fs / (d * u.x);
  }
  return u;
}

// Pair t (0-based, p < q, row by row) of K users.
__device__ __forceinline__ void pair_of(int K, int t, int& p, int& q) {
  p = 0;
  int rem = t;
  while (rem >= K - 1 - p) {
    rem -= K - 1 - p;
    ++p;
  }
  q = p + 1 + rem;
}

// Per-pair word written by k_cf_pairs for the per-drop pass: route in bits 0-1,
// degenerate pair (GATED entry with x_i == x_j) in bit 2, panels from bit 3.
constexpr int kPairDegenerate = 4;

// GATED entry of an analytic ULA pair: the stationary-phase term (eq. (6) or its
// free-space analogue), zero with the stationary point off the aperture.
__device__ __forceinline__ Cplx gated_ula(const ArrayK& arr, const UlaUser& up, const UlaUser& uq, double Ly,
                                          double c_fs, bool& degenerate) {
  const double d = arr.spacing, lam = arr.lambda;
  const double xp = up.x, xq = uq.x;
  const double dx = xp - xq, dy = up.y - uq.y;
  const double dist = sqrt(dx * dx + dy * dy);
  degenerate = false;
  if (dx == 0.0 || dist == 0.0) {
    degenerate = true;
    return Cplx{0.0, 0.0};
  }
  if (!(fabs((up.y * xq - xp * uq.y) / (xq - xp)) <= Ly)) return Cplx{0.0, 0.0};
  const double sg = dx > 0.0 ? 1.0 : -1.0;
  double mag;
  if (arr.amp == XLMIMO_AMP_PNUSW) {
    const double rho = sqrt(lam) * fabs(dx) / (dist * sqrt(dist)) / sqrt(up.sfac * uq.sfac);
    mag = rho * sqrt(up.diag * uq.diag);
  } else {
    mag = c_fs * sqrt(lam) / (d * sqrt(xp * xq * dist));
  }
  double tt;
  int qd;
  reduce_quarter(dist * arr.inv_lambda - 0.125, tt, qd);
  double sn, cs, cre, cim;
  sincos_rev(tt, sn, cs);
  rotate_conj(1.0, sn, cs, qd, cre, cim);
  return Cplx{mag * cre, -sg * mag * cim};
}

// Analytic pairs of the ULA variants UNIFORM and GATED_QUAD, one thread per pair over the
// whole batch (the drop found by bisection of the pairs' offsets).  Writes the entry and its
// conjugate for analytic pairs and NaN for pairs with a bad user; records every pair's route
// for k_closedform, which evaluates the numeric ones.  Lanes past the last pair stay in the
// wave (idle) until the Fresnel integrals of the uniform form have been completed together.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_cf_pairs(ArrayK arr, const DropK* __restrict__ drops, int n_drops,
                                                  int64_t n_pairs, int variant, const double* __restrict__ pos,
                                                  const double* __restrict__ gl, int n_gl,
                                                  double* __restrict__ gram, int32_t* __restrict__ route_out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < n_pairs;
  FresnelReq fr;
  fr.need[0] = fr.need[1] = false;
  Cplx v = {0.0, 0.0};
  bool write = false;
  int K = 0, p = 0, q = 0, word = ROUTE_NONE;
  double* out = gram;
  if (valid) {
    int lo = 0, hi = n_drops - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (drops[mid].pair_off <= t) lo = mid;
      else hi = mid - 1;
    }
    const DropK dp = drops[lo];
    K = dp.k;
    pair_of(K, (int)(t - dp.pair_off), p, q);
    const double d = arr.spacing, lam = arr.lambda;
    const double c_fs = (lam / (4.0 * kPi)) * (lam / (4.0 * kPi));
    const double Ly = 0.5 * (double)dp.n_elems * d;
    // no closed-form diagonal is read here (k_closedform writes it): only its finiteness
    const UlaUser up = ula_user(arr, pos + (dp.user_off + p) * 3, Ly, c_fs, false);
    const UlaUser uq = ula_user(arr, pos + (dp.user_off + q) * 3, Ly, c_fs, false);
    out = gram + 2 * dp.gram_off;
    write = true;
    if (!(up.ok && uq.ok && isfinite(up.diag) && isfinite(uq.diag))) {
      v = Cplx{__builtin_nan(""), __builtin_nan("")};
    } else {
      const PairGeom g{up.x, up.y, uq.x, uq.y, 2.0 * kPi * arr.inv_lambda, arr.inv_lambda, arr.amp, arr.beta0, c_fs};
      int panels = 0;
      const int route = numeric_route(g, dp.n_elems, d, n_gl, panels);
      if (route != ROUTE_NONE) {
        word = route | (panels << 3);
        write = false;   // k_closedform evaluates it
      } else if (variant == XLMIMO_CF_UNIFORM) {
        v = uniform_pair(g, dp.n_elems, d, fr);
      } else {
        bool degenerate;
        v = gated_ula(arr, up, uq, Ly, c_fs, degenerate);
        if (degenerate) word |= kPairDegenerate;
      }
    }
  }
  fresnel_complete(fr, v, gl + 2 * n_gl);   // the Fresnel rule follows the n_gl-node one
  if (!valid) return;
  route_out[t] = word;
  if (write) {
    out[2 * (p * K + q)] = v.re;
    out[2 * (p * K + q) + 1] = v.im;
    out[2 * (q * K + p)] = v.re;
    out[2 * (q * K + p) + 1] = -v.im;
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_closedform(ArrayK arr, const DropK* __restrict__ drops, int variant,
                                                     const double* __restrict__ pos,
                                                     const double* __restrict__ gl, int n_gl,
                                                     double* __restrict__ gram, int32_t* __restrict__ status,
                                                     const int32_t* __restrict__ route_in) {
  __shared__ double s_x[XLMIMO_MAX_USERS], s_y[XLMIMO_MAX_USERS], s_z[XLMIMO_MAX_USERS];
  __shared__ double s_diag[XLMIMO_MAX_USERS], s_sfac[XLMIMO_MAX_USERS];
  __shared__ int s_status;
  const DropK dp = drops[blockIdx.x];
  const int K = dp.k;
  const double d = arr.spacing, lam = arr.lambda;
  const double c_fs = (lam / (4.0 * kPi)) * (lam / (4.0 * kPi));
  const bool ula = arr.geom == XLMIMO_ULA;
  const double Ly = 0.5 * (double)(ula ? dp.n_elems : arr.n_y) * d;
  const double Lz = 0.5 * (double)arr.n_z * d;
  if (threadIdx.x == 0) s_status = 0;
  __syncthreads();

  for (int i = threadIdx.x; i < K; i += blockDim.x) {
    const double* p = pos + (dp.user_off + i) * 3;
    const double px = p[0], py = p[1], pz = p[2];
    const double x = ula ? sqrt(fma(px, px, pz * pz)) : fabs(px);
    s_x[i] = x;
    s_y[i] = py;
    s_z[i] = pz;
    double g = 0.0, sf = 0.0;
    const bool ok = x > 0.0 && isfinite(x) && isfinite(py) && isfinite(pz);
    if (!ok) {
      atomicOr(&s_status, XLMIMO_ST_BAD_INPUT);
      g = __builtin_nan("");
    } else if (ula) {
      if (arr.amp == XLMIMO_AMP_PNUSW) {
        const double a = Ly - py, b = Ly + py;
        sf = a / sqrt(fma(a, a, x * x)) + b / sqrt(fma(b, b, x * x));
        g = arr.beta0 / (d * x) * sf;
      } else {
        g = c_fs / (d * x) * (atan((Ly - py) / x) + atan((Ly + py) / x));
      }
    } else {
      if (arr.amp == XLMIMO_AMP_PNUSW) {
        g = arr.beta0 / (d * d) * solid_angle_rect(x, -Ly - py, Ly - py, -Lz - pz, Lz - pz);
      } else {
        g = c_fs / (d * d) * upa_freespace_integral(x, -Ly - py, Ly - py, -Lz - pz, Lz - pz, gl, n_gl);
      }
    }
    s_diag[i] = g;
    s_sfac[i] = sf;
  }
  __syncthreads();

  double* out = gram + 2 * dp.gram_off;
  if (ula && (variant == XLMIMO_CF_UNIFORM || variant == XLMIMO_CF_GATED_QUAD)) {
    // The diagonal, then the numeric pairs (slow-phase pairs, broad stationary zones) queued from
    // k_cf_pairs' route words: direct sums and quadratures by the whole workgroup.
    __shared__ int s_nq, s_nd;
    __shared__ __align__(16) int s_queue[XLMIMO_MAX_USERS * (XLMIMO_MAX_USERS - 1) / 2][3];  // pair, route, panels
    if (threadIdx.x == 0) s_nq = s_nd = 0;
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
      out[2 * (i * K + i)] = s_diag[i];
      out[2 * (i * K + i) + 1] = 0.0;
    }
    __syncthreads();
    const int np = K * (K - 1) / 2;
    const int n = dp.n_elems;
    const double kw = 2.0 * kPi * arr.inv_lambda;
    auto pair_of_k = [K](int t, int& p, int& q) { pair_of(K, t, p, q); };
    // analytic pairs were written by k_cf_pairs; queue the numeric ones from its route words
    const int32_t* rw = route_in + dp.pair_off;
    for (int t = threadIdx.x; t < np; t += blockDim.x) {
      const int w = rw[t];
      if (w & kPairDegenerate) atomicOr(&s_status, XLMIMO_ST_CF_DEGENERATE);
      const int route = w & 3;
      if (route != ROUTE_NONE) {
        const int slot = atomicAdd(&s_nq, 1);
        if (route == ROUTE_DIRECT) atomicAdd(&s_nd, 1);
        s_queue[slot][0] = t;
        s_queue[slot][1] = route;
        s_queue[slot][2] = w >> 3;
      }
    }
    __syncthreads();
    const int nq = s_nq;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    const int nd = s_nd;
    const bool shared_chan = 2 * nd > K && nd <= (int)blockDim.x && nd == nq;
    if (shared_chan) {
      // Many direct sums and nothing else numeric (always so for N <= kDirectMaxN): each user's channel
      // h_u(y) = a_u(r) e^{-j 2 pi r / lambda} is formed once per element chunk in LDS (over the queue,
      // whose pairs are copied out first) and every direct pair sums conj(h_p) h_q from there.  A pair's
      // elements are split into `sub` interleaved partial sums (a fixed split for the drop), combined in
      // order.
      constexpr int kChan = (int)sizeof(s_queue) / (2 * (int)sizeof(double));
      double* s_h = reinterpret_cast<double*>(&s_queue[0][0]);
      __shared__ double s_part[2 * 256];
      __shared__ int s_dl[256];
      for (int e = threadIdx.x; e < nq; e += blockDim.x) s_dl[e] = s_queue[e][0];
      int sub = 1;
      while (2 * sub * nd <= (int)blockDim.x && sub < 64) sub *= 2;
      const int chunk = kChan / K;
      const double sq_fs = sqrt(c_fs);
      __syncthreads();
      const int me = threadIdx.x / sub, ms = threadIdx.x % sub;
      int p = 0, q = 0;
      if (me < nd) pair_of_k(s_dl[me], p, q);
      Cplx acc = {0.0, 0.0};
      for (int n0 = 0; n0 < n; n0 += chunk) {
        const int cn = min(chunk, n - n0);
        for (int idx = threadIdx.x; idx < K * cn; idx += blockDim.x) {
          const int u = idx / cn, e = idx - u * cn;
          const double y = ((double)(n0 + e) - 0.5 * (double)(n - 1)) * d;
          const double dy = y - s_y[u], x = s_x[u];
          double r, ir;
          dist_inv(fma(dy, dy, x * x), r, ir);
          const double a = arr.amp == XLMIMO_AMP_PNUSW ? sqrt(arr.beta0 * x) * ir * sqrt(ir) : sq_fs * ir;
          const Cplx ph = phasor_turns_d(r * arr.inv_lambda);
          s_h[2 * (u * chunk + e)] = a * ph.re;
          s_h[2 * (u * chunk + e) + 1] = -a * ph.im;
        }
        __syncthreads();
        if (me < nd) {
          const double* hp = s_h + 2 * p * chunk;
          const double* hq = s_h + 2 * q * chunk;
          for (int e = ms; e < cn; e += sub) {
            // conj(h_p) h_q
            const double pr = hp[2 * e], pi = hp[2 * e + 1], qr = hq[2 * e], qi = hq[2 * e + 1];
            acc.re += pr * qr + pi * qi;
            acc.im += pr * qi - pi * qr;
          }
        }
        __syncthreads();
      }
      if (me < nd) {
        s_part[2 * threadIdx.x] = acc.re;
        s_part[2 * threadIdx.x + 1] = acc.im;
      }
      __syncthreads();
      if ((int)threadIdx.x < nd) {
        int pp, qq;
        pair_of_k(s_dl[threadIdx.x], pp, qq);
        Cplx v = {0.0, 0.0};
        for (int m = 0; m < sub; ++m) v = cadd(v, Cplx{s_part[2 * (threadIdx.x * sub + m)], s_part[2 * (threadIdx.x * sub + m) + 1]});
        out[2 * (pp * K + qq)] = v.re;
        out[2 * (pp * K + qq) + 1] = v.im;
        out[2 * (qq * K + pp)] = v.re;
        out[2 * (qq * K + pp) + 1] = -v.im;
      }
    }
    // otherwise: direct sums one wave per pair, fixed-order wave sum
    for (int e = wave; e < nq && !shared_chan; e += n_waves) {
      if (s_queue[e][1] != ROUTE_DIRECT) continue;
      int p, q;
      pair_of_k(s_queue[e][0], p, q);
      const PairGeom g{s_x[p], s_y[p], s_x[q], s_y[q], kw, arr.inv_lambda, arr.amp, arr.beta0, c_fs};
      const Cplx v = wave_sum_c(numeric_share(g, n, d, ROUTE_DIRECT, 0, gl, n_gl, lane, 64));
      if (lane == 0) {
        out[2 * (p * K + q)] = v.re;
        out[2 * (p * K + q) + 1] = v.im;
        out[2 * (q * K + p)] = v.re;
        out[2 * (q * K + p) + 1] = -v.im;
      }
    }
    // quadratures (up to N/4 nodes), one pair at a time: every thread takes a share of the nodes;
    // wave sums, then the waves' sums in order
    __shared__ double s_wsum[2 * 16];
    for (int e = 0; e < nq && !shared_chan; ++e) {
      const int t = s_queue[e][0], route = s_queue[e][1], panels = s_queue[e][2];
      if (route != ROUTE_QUAD) continue;
      int p, q;
      pair_of_k(t, p, q);
      const PairGeom g{s_x[p], s_y[p], s_x[q], s_y[q], kw, arr.inv_lambda, arr.amp, arr.beta0, c_fs};
      const Cplx v = wave_sum_c(numeric_share(g, n, d, route, panels, gl, n_gl, threadIdx.x, blockDim.x));
      if (lane == 0) {
        s_wsum[2 * wave] = v.re;
        s_wsum[2 * wave + 1] = v.im;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        Cplx tot = {0.0, 0.0};
        for (int w = 0; w < n_waves; ++w) tot = cadd(tot, Cplx{s_wsum[2 * w], s_wsum[2 * w + 1]});
        tot = cadd(cscale(tot, 1.0 / d), discrete_end_corrections(g, n, d));
        out[2 * (p * K + q)] = tot.re;
        out[2 * (p * K + q) + 1] = tot.im;
        out[2 * (q * K + p)] = tot.re;
        out[2 * (q * K + p) + 1] = -tot.im;
      }
      __syncthreads();
    }
    if (status != nullptr && threadIdx.x == 0) status[blockIdx.x] = s_status;
    return;
  }
  for (int idx = threadIdx.x; idx < K * K; idx += blockDim.x) {
    const int i = idx / K, j = idx - (idx / K) * K;
    double re = 0.0, im = 0.0;
    if (i == j) {
      re = s_diag[i];
    } else {
      const int p = i < j ? i : j, q = i < j ? j : i;  // compute (p, q), conjugate for i > j
      const double xp = s_x[p], xq = s_x[q];
      const double dx = xp - xq, dy = s_y[p] - s_y[q], dz = ula ? 0.0 : s_z[p] - s_z[q];
      const double dist = sqrt(dx * dx + dy * dy + dz * dz);
      if (!(isfinite(s_diag[p]) && isfinite(s_diag[q]))) {
        re = im = __builtin_nan("");
      } else if (dx == 0.0 || dist == 0.0) {
        if (i < j) atomicOr(&s_status, XLMIMO_ST_CF_DEGENERATE);
      } else {
        bool inside = true;
        if (variant == XLMIMO_CF_GATED) {
          const double ys = (s_y[p] * xq - xp * s_y[q]) / (xq - xp);
          inside = fabs(ys) <= Ly;
          if (!ula) {
            const double zs = (s_z[p] * xq - xp * s_z[q]) / (xq - xp);
            inside = inside && fabs(zs) <= Lz;
          }
        }
        if (inside) {
          const double sg = dx > 0.0 ? 1.0 : -1.0;
          double mag, off;
          if (ula) {
            off = 0.125;  // pi/4 in revolutions
            if (arr.amp == XLMIMO_AMP_PNUSW) {
              const double rho = sqrt(lam) * fabs(dx) / (dist * sqrt(dist)) / sqrt(s_sfac[p] * s_sfac[q]);
              mag = rho * sqrt(s_diag[p] * s_diag[q]);
            } else {
              mag = c_fs * sqrt(lam) / (d * sqrt(xp * xq * dist));
            }
          } else {
            off = 0.25;  // pi/2 in revolutions
            mag = (arr.amp == XLMIMO_AMP_PNUSW) ? arr.beta0 * lam / (d * d * dist) : c_fs * lam / (d * d * fabs(dx));
          }
          double t;
          int qd;
          reduce_quarter(dist * arr.inv_lambda - off, t, qd);
          double s, c, cre, cim;
          sincos_rev(t, s, c);
          rotate_conj(1.0, s, c, qd, cre, cim);  // (cos phi, -sin phi), phi = 2 pi (d/lambda - off)
          re = mag * cre;
          im = -sg * mag * cim;                  // e^{j s phi}
        }
      }
      if (i > j) im = -im;
    }
    out[2 * idx] = re;
    out[2 * idx + 1] = im;
  }
  __syncthreads();
  if (status != nullptr && threadIdx.x == 0) status[blockIdx.x] = s_status;
}

hipError_t launch_closedform(const ArrayK& arr, const DropK* d_drops, int n_drops, int variant, const double* d_pos,
                             const double* d_gl, int n_gl, double* d_diag, double* d_gram, int32_t* d_status,
                             int k_max, hipStream_t s, int64_t n_pairs, int32_t* d_route) {
  (void)d_diag;
  (void)k_max;
  if (n_drops == 0) return hipSuccess;
  const bool split = arr.geom == XLMIMO_ULA && (variant == XLMIMO_CF_UNIFORM || variant == XLMIMO_CF_GATED_QUAD);
  if (split) {
    if (d_route == nullptr) return hipErrorInvalidValue;
    if (n_pairs > 0)
      k_cf_pairs<<<(unsigned)((n_pairs + 255) / 256), 256, 0, s>>>(arr, d_drops, n_drops, n_pairs, variant, d_pos, d_gl,
                                                                  n_gl, d_gram, d_route);
  }
  k_closedform<<<n_drops, 256, 0, s>>>(arr, d_drops, variant, d_pos, d_gl, n_gl, d_gram, d_status, d_route);
  return hipGetLastError();
}

}  // namespace xl
