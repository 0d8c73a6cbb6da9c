// Sweep epilogues: ergodic means over drops and the saturation point.
//
// Sec. IV-C verifies the saturation point on ergodic capacity-vs-M curves.
//   * ergodic mean: for every (SNR, scheme) value, the mean over drops whose
//     rate is finite (a closed-form Gram may be indefinite at small N).
//   * analytic saturation: per drop y_up = max_i (tau x_i + y_i) and
//     y_down = min_i (-tau x_i + y_i), tau = t / sqrt(1 - t^2) (eqs. (13)-(16));
//     their means over drops give M_sat = (E[y_up] - E[y_down]) / spacing.
//   * empirical saturation: first N, interpolated linearly in log N, where the
//     ergodic curve reaches (1 - eps) of its value at the largest N.
// Reductions are fixed-order trees, so results are repeatable.
#include "internal.h"
#include "xlmimo.h"

namespace xl {

__device__ __forceinline__ void block_sum2(double& a, double& b, double* sa, double* sb) {
  const int t = threadIdx.x;
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (t < off) {
      sa[t] += sa[t + off];
      sb[t] += sb[t + off];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_ergodic(const double* __restrict__ rates, int n_drops, int n_vals,
                                                 double* __restrict__ out) {
  __shared__ double sa[256], sb[256];
  const int v = blockIdx.x;
  double sum = 0.0, cnt = 0.0;
  for (int d = threadIdx.x; d < n_drops; d += blockDim.x) {
    const double r = rates[(int64_t)d * n_vals + v];
    if (isfinite(r)) {
      sum += r;
      cnt += 1.0;
    }
  }
  block_sum2(sum, cnt, sa, sb);
  if (threadIdx.x == 0) out[v] = cnt > 0.0 ? sum / cnt : __builtin_nan("");
}

__global__ void k_y_bounds(const double* __restrict__ pos, const DropK* __restrict__ drops, int n_drops, int geom,
                           double tau, double* __restrict__ bounds) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n_drops) return;
  const DropK dp = drops[d];
  double up = -INFINITY, dn = INFINITY;
  for (int i = 0; i < dp.k; ++i) {
    const double* p = pos + (dp.user_off + i) * 3;
    const double x = (geom == XLMIMO_ULA) ? sqrt(fma(p[0], p[0], p[2] * p[2])) : fabs(p[0]);
    up = fmax(up, fma(tau, x, p[1]));
    dn = fmin(dn, fma(-tau, x, p[1]));
  }
  bounds[2 * d] = up;
  bounds[2 * d + 1] = dn;
}

__global__ __launch_bounds__(256) void k_saturation(const double* __restrict__ bounds, int n_drops,
                                                    const double* __restrict__ ergodic,
                                                    const double* __restrict__ nlist, int n_N, int n_vals,
                                                    double spacing, double eps, double* __restrict__ sat) {
  __shared__ double sa[256], sb[256];
  double up = 0.0, dn = 0.0;
  for (int d = threadIdx.x; d < n_drops; d += blockDim.x) {
    up += bounds[2 * d];
    dn += bounds[2 * d + 1];
  }
  block_sum2(up, dn, sa, sb);
  if (threadIdx.x == 0) {
    const double eu = up / n_drops, ed = dn / n_drops;
    sat[0] = eu;
    sat[1] = ed;
    sat[2] = (eu - ed) / spacing;
  }
  for (int v = threadIdx.x; v < n_vals; v += blockDim.x) {
    const double cmax = ergodic[(int64_t)(n_N - 1) * n_vals + v];
    const double target = 1.0 - eps;
    double res = nlist[n_N - 1];
    for (int n = 0; n < n_N; ++n) {
      const double c = ergodic[(int64_t)n * n_vals + v] / cmax;
      if (c >= target) {
        if (n == 0) {
          res = nlist[0];
        } else {
          const double cp = ergodic[(int64_t)(n - 1) * n_vals + v] / cmax;
          const double f = (target - cp) / (c - cp);
          res = exp(log(nlist[n - 1]) + f * (log(nlist[n]) - log(nlist[n - 1])));
        }
        break;
      }
    }
    sat[3 + v] = res;
  }
}

hipError_t launch_ergodic(const double* d_rates, int n_drops, int n_vals, double* d_out, hipStream_t s) {
  k_ergodic<<<n_vals, 256, 0, s>>>(d_rates, n_drops, n_vals, d_out);
  return hipGetLastError();
}

hipError_t launch_y_bounds(const double* d_pos, const DropK* d_drops, int n_drops, int geom, double t_sat,
                           double* d_bounds, hipStream_t s) {
  const double tau = t_sat / sqrt(1.0 - t_sat * t_sat);
  k_y_bounds<<<(n_drops + 255) / 256, 256, 0, s>>>(d_pos, d_drops, n_drops, geom, tau, d_bounds);
  return hipGetLastError();
}

hipError_t launch_saturation(const double* d_bounds, int n_drops, const double* d_ergodic, const double* d_nlist,
                             int n_N, int n_vals, double spacing, double eps, double* d_sat, hipStream_t s) {
  k_saturation<<<1, 256, 0, s>>>(d_bounds, n_drops, d_ergodic, d_nlist, n_N, n_vals, spacing, eps, d_sat);
  return hipGetLastError();
}

}  // namespace xl
