// Linear-receiver sum-rates of a batch of drops from their K x K Grams, FP64.
//
// The paper fixes the capacity (eq. (9)) and the ZF equaliser (eq. (21)); the
// per-user SINRs are the textbook ones (rho_k = P_k / sigma^2, D = diag(rho),
// A = D^1/2 G D^1/2):
//   ZF    rho_k / [G^-1]_kk                  MMSE  1 / [(I + A)^-1]_kk - 1
//   MRC   rho_k G_kk^2 / (sum_{j!=k} rho_j |G_kj|^2 + G_kk)
//   CAP   log2 det(I + A)                     MZF   rho_k / [G~^-1]_kk
//   MZF_MISM  B = G~^-1 G:  rho_k |B_kk|^2 / (sum_{j!=k} rho_j |B_kj|^2 + [G~^-1 G G~^-1]_kk)
//
// One 64-lane wave per drop (K <= 64: lane i owns row i / column i).  The
// Hermitian matrix is factorised in LDS by a right-looking Cholesky G = L L^H
// (lower triangle); W = L^-1 is formed by forward substitution with lane k
// solving column k and storing W_ik (i > k) in the unused upper triangle, so
// [G^-1]_kk = sum_i |W_ik|^2.  log det = 2 sum log L_kk.  A non-positive or
// non-finite pivot marks the drop (XLMIMO_ST_*) and yields NaN rates.
// Sums over users use a fixed butterfly order, so results are repeatable.
#include "internal.h"
#include "xlmimo.h"

namespace xl {

struct cplx {
  double x, y;
};

__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cplx cmulc(cplx a, cplx b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
__device__ __forceinline__ cplx cconjmul(cplx a, cplx b) {  // conj(a) * b
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Cholesky of the K x K Hermitian matrix in A (row stride ld), lower triangle.
__device__ bool chol_lower(cplx* A, int K, int ld, int lane) {
  for (int j = 0; j < K; ++j) {
    const double djj = A[j * ld + j].x;
    __syncthreads();
    if (!(djj > 0.0) || !isfinite(djj)) return false;  // uniform: every lane read the same pivot
    const double l = sqrt(djj), il = 1.0 / l;
    if (lane > j && lane < K) {
      cplx v = A[lane * ld + j];
      A[lane * ld + j] = {v.x * il, v.y * il};
    }
    if (lane == j) A[j * ld + j] = {l, 0.0};
    __syncthreads();
    if (lane > j && lane < K) {
      const cplx lij = A[lane * ld + j];
      for (int c = j + 1; c <= lane; ++c) {
        const cplx t = cmulc(lij, A[c * ld + j]);
        cplx v = A[lane * ld + c];
        A[lane * ld + c] = {v.x - t.x, v.y - t.y};
      }
    }
    __syncthreads();
  }
  return true;
}

// W = L^-1, column `lane` stored at A[lane * ld + i] (i > lane) and wd[lane];
// returns [ (L L^H)^-1 ]_{lane,lane} = sum_i |W_{i,lane}|^2.
__device__ double inverse_diag(cplx* A, double* wd, int K, int ld, int lane) {
  double s = 0.0;
  if (lane < K) {
    const double w0 = 1.0 / A[lane * ld + lane].x;
    wd[lane] = w0;
    s = w0 * w0;
    for (int i = lane + 1; i < K; ++i) {
      cplx acc = {A[i * ld + lane].x * w0, A[i * ld + lane].y * w0};
      for (int m = lane + 1; m < i; ++m) {
        const cplx t = cmul(A[i * ld + m], A[lane * ld + m]);
        acc.x += t.x;
        acc.y += t.y;
      }
      const double il = -1.0 / A[i * ld + i].x;
      const cplx w = {acc.x * il, acc.y * il};
      A[lane * ld + i] = w;
      s += w.x * w.x + w.y * w.y;
    }
  }
  __syncthreads();
  return s;
}

__device__ __forceinline__ cplx gload(const double* g, int64_t off, int K, int i, int j) {
  const double* p = g + 2 * (off + (int64_t)i * K + j);
  return {p[0], p[1]};
}

__global__ __launch_bounds__(64) void k_rates(const DropK* __restrict__ drops, const double* __restrict__ gram,
                                              const double* __restrict__ filter, int n_snr,
                                              const double* __restrict__ rho, int64_t total_users, int schemes,
                                              int n_sch, double* __restrict__ rates, int32_t* __restrict__ status,
                                              int ld) {
  extern __shared__ double smem[];
  const bool mism = schemes & XLMIMO_MZF_MISM;
  cplx* A = reinterpret_cast<cplx*>(smem);
  const int rows = ld - 1;
  cplx* Q = A + rows * ld;                                // used by MZF_MISM only
  double* wd = reinterpret_cast<double*>(A + (mism ? 2 : 1) * rows * ld);
  const int lane = threadIdx.x;
  const DropK dp = drops[blockIdx.x];
  const int K = dp.k;
  const int64_t go = dp.gram_off;
  int st = 0;
  const double nan = __builtin_nan("");

  // ZF: [G^-1]_kk (independent of the SNR)
  double ginv = nan;
  if (schemes & XLMIMO_ZF) {
    if (lane < K)
      for (int j = 0; j < K; ++j) A[lane * ld + j] = gload(gram, go, K, lane, j);
    __syncthreads();
    if (chol_lower(A, K, ld, lane)) ginv = inverse_diag(A, wd, K, ld, lane);
    else st |= XLMIMO_ST_G_NOT_PD;
    __syncthreads();
  }

  // Modified ZF on the filter Gram: nominal [G~^-1]_kk, and the mismatched terms.
  double finv = nan, noise = nan, bkk2 = nan;
  if (schemes & (XLMIMO_MZF | XLMIMO_MZF_MISM)) {
    if (lane < K)
      for (int j = 0; j < K; ++j) A[lane * ld + j] = gload(filter, go, K, lane, j);
    __syncthreads();
    bool ok = chol_lower(A, K, ld, lane);
    if (ok) {
      finv = inverse_diag(A, wd, K, ld, lane);
    } else {
      st |= XLMIMO_ST_FILTER_NOT_PD;
    }
    if (ok && mism) {
      // Q = G~^-1 = W^H W, row `lane`: Q_kj = sum_{i >= max(k,j)} conj(W_ik) W_ij
      if (lane < K) {
        for (int j = 0; j < K; ++j) {
          cplx acc = {0.0, 0.0};
          const int i0 = lane > j ? lane : j;
          for (int i = i0; i < K; ++i) {
            const cplx wik = (i == lane) ? cplx{wd[lane], 0.0} : A[lane * ld + i];
            const cplx wij = (i == j) ? cplx{wd[j], 0.0} : A[j * ld + i];
            const cplx t = cconjmul(wik, wij);
            acc.x += t.x;
            acc.y += t.y;
          }
          Q[lane * ld + j] = acc;
        }
      }
      __syncthreads();
      // B = Q G (true Gram); |B_kj|^2 kept in A's real parts; noise_k = sum_j B_kj Q_jk
      if (lane < K) {
        double nz = 0.0;
        for (int j = 0; j < K; ++j) {
          cplx b = {0.0, 0.0};
          for (int m = 0; m < K; ++m) {
            const cplx t = cmul(Q[lane * ld + m], gload(gram, go, K, m, j));
            b.x += t.x;
            b.y += t.y;
          }
          const cplx t = cmulc(b, Q[lane * ld + j]);  // B_kj * Q_jk, Q_jk = conj(Q_kj)
          nz += t.x;
          A[lane * ld + j] = {b.x * b.x + b.y * b.y, 0.0};
        }
        noise = nz;
        bkk2 = A[lane * ld + lane].x;
      }
    }
    __syncthreads();
  }

  // MMSE works in Q when the mismatched scheme keeps |B_kj|^2 in A.
  cplx* M = mism ? Q : A;
  const int64_t rbase = (int64_t)blockIdx.x * n_snr * n_sch;
  for (int s = 0; s < n_snr; ++s) {
    const double* rs = rho + (int64_t)s * total_users + dp.user_off;
    const double rk = lane < K ? rs[lane] : 0.0;
    int c = 0;
    if (schemes & XLMIMO_ZF) {
      const double v = lane < K ? log2(1.0 + rk / ginv) : 0.0;
      const double tot = wave_sum(v);
      if (lane == 0) rates[rbase + s * n_sch + c] = tot;
      ++c;
    }
    if (schemes & (XLMIMO_MMSE | XLMIMO_CAP)) {
      __syncthreads();
      if (lane < K) {
        const double sk = sqrt(rk);
        for (int j = 0; j < K; ++j) {
          const cplx g = gload(gram, go, K, lane, j);
          const double sj = sqrt(rs[j]);
          M[lane * ld + j] = {(lane == j ? 1.0 : 0.0) + sk * sj * g.x, sk * sj * g.y};
        }
      }
      __syncthreads();
      double mmse = nan, cap = nan;
      if (chol_lower(M, K, ld, lane)) {
        const double logd = wave_sum(lane < K ? log2(M[lane * ld + lane].x) : 0.0);
        cap = 2.0 * logd;
        const double minv = inverse_diag(M, wd, K, ld, lane);
        mmse = wave_sum(lane < K ? -log2(minv) : 0.0);   // log2(1 + SINR) = -log2 [M^-1]_kk
      } else {
        st |= XLMIMO_ST_MMSE_NOT_PD;
      }
      if (schemes & XLMIMO_MMSE) {
        if (lane == 0) rates[rbase + s * n_sch + c] = mmse;
        ++c;
      }
      if (schemes & XLMIMO_MRC) {
        double v = 0.0;
        if (lane < K) {
          const double gkk = gload(gram, go, K, lane, lane).x;
          double interf = 0.0;
          for (int j = 0; j < K; ++j) {
            if (j == lane) continue;
            const cplx g = gload(gram, go, K, lane, j);
            interf += rs[j] * (g.x * g.x + g.y * g.y);
          }
          v = log2(1.0 + rk * gkk * gkk / (interf + gkk));
        }
        const double tot = wave_sum(v);
        if (lane == 0) rates[rbase + s * n_sch + c] = tot;
        ++c;
      }
      if (schemes & XLMIMO_CAP) {
        if (lane == 0) rates[rbase + s * n_sch + c] = cap;
        ++c;
      }
    } else if (schemes & XLMIMO_MRC) {
      double v = 0.0;
      if (lane < K) {
        const double gkk = gload(gram, go, K, lane, lane).x;
        double interf = 0.0;
        for (int j = 0; j < K; ++j) {
          if (j == lane) continue;
          const cplx g = gload(gram, go, K, lane, j);
          interf += rs[j] * (g.x * g.x + g.y * g.y);
        }
        v = log2(1.0 + rk * gkk * gkk / (interf + gkk));
      }
      const double tot = wave_sum(v);
      if (lane == 0) rates[rbase + s * n_sch + c] = tot;
      ++c;
    }
    if (schemes & XLMIMO_MZF) {
      const double tot = wave_sum(lane < K ? log2(1.0 + rk / finv) : 0.0);
      if (lane == 0) rates[rbase + s * n_sch + c] = tot;
      ++c;
    }
    if (schemes & XLMIMO_MZF_MISM) {
      double v = 0.0;
      if (lane < K) {
        double interf = 0.0;
        for (int j = 0; j < K; ++j)
          if (j != lane) interf += rs[j] * A[lane * ld + j].x;
        v = log2(1.0 + rk * bkk2 / (interf + noise));
      }
      const double tot = wave_sum(v);
      if (lane == 0) rates[rbase + s * n_sch + c] = tot;
      ++c;
    }
  }
  if (status != nullptr && lane == 0) status[blockIdx.x] = st;
}

hipError_t launch_rates(const DropK* d_drops, int n_drops, int k_max, const double* d_gram, const double* d_filter,
                        int n_snr, const double* d_rho, int64_t total_users, int schemes, double* d_rates,
                        int32_t* d_status, hipStream_t s) {
  if (n_drops == 0) return hipSuccess;
  int n_sch = __builtin_popcount(schemes);
  const int ld = k_max + 1;
  const bool mism = schemes & XLMIMO_MZF_MISM;
  const size_t lds = (size_t)(mism ? 2 : 1) * k_max * ld * sizeof(cplx) + 64 * sizeof(double);
  k_rates<<<n_drops, 64, lds, s>>>(d_drops, d_gram, d_filter, n_snr, d_rho, total_users, schemes, n_sch, d_rates,
                                    d_status, ld);
  return hipGetLastError();
}

}  // namespace xl
