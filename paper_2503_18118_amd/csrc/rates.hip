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

// Q = A^-1 by Gauss-Jordan elimination with partial pivoting (A is overwritten),
// lane i owning row i.  The pivot is the largest |A_ic|, i >= c, by a fixed-order
// wave reduction (ties to the lower row), so results are repeatable.  Returns
// false (uniformly) for a zero or non-finite pivot.  Used for the mismatched
// modified ZF when the filter Gram is not positive definite: the filter
// G~^-1 H^H needs G~ invertible, not definite.
__device__ bool gauss_jordan_inverse(cplx* A, cplx* Q, int K, int ld, int lane) {
  if (lane < K)
    for (int j = 0; j < K; ++j) Q[lane * ld + j] = {lane == j ? 1.0 : 0.0, 0.0};
  __syncthreads();
  for (int c = 0; c < K; ++c) {
    double mag = -1.0;
    int idx = lane;
    if (lane >= c && lane < K) {
      const cplx v = A[lane * ld + c];
      mag = v.x * v.x + v.y * v.y;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double om = __shfl_xor(mag, off, 64);
      const int oi = __shfl_xor(idx, off, 64);
      if (om > mag || (om == mag && oi < idx)) {
        mag = om;
        idx = oi;
      }
    }
    if (!(mag > 0.0) || !isfinite(mag)) return false;  // uniform: every lane holds the same maximum
    const int pr = idx;
    if (pr != c && lane < K) {
      const cplx ta = A[c * ld + lane], tq = Q[c * ld + lane];
      A[c * ld + lane] = A[pr * ld + lane];
      Q[c * ld + lane] = Q[pr * ld + lane];
      A[pr * ld + lane] = ta;
      Q[pr * ld + lane] = tq;
    }
    __syncthreads();
    const cplx pv = A[c * ld + c];
    const double den = pv.x * pv.x + pv.y * pv.y;
    const cplx ip = {pv.x / den, -pv.y / den};
    __syncthreads();  // every lane has read the pivot before row c changes
    if (lane < K) {
      A[c * ld + lane] = cmul(A[c * ld + lane], ip);
      Q[c * ld + lane] = cmul(Q[c * ld + lane], ip);
    }
    __syncthreads();
    if (lane < K && lane != c) {
      const cplx f = A[lane * ld + c];
      for (int j = 0; j < K; ++j) {
        const cplx ta = cmul(f, A[c * ld + j]), tq = cmul(f, Q[c * ld + j]);
        A[lane * ld + j] = {A[lane * ld + j].x - ta.x, A[lane * ld + j].y - ta.y};
        Q[lane * ld + j] = {Q[lane * ld + j].x - tq.x, Q[lane * ld + j].y - tq.y};
      }
    }
    __syncthreads();
  }
  return true;
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

  // ZF: [G^-1]_kk; the correlation gap -(1/K) log2 det R from the same factor (both independent of
  // the SNR)
  double ginv = nan, gapv = nan;
  if (schemes & (XLMIMO_ZF | XLMIMO_CORR_GAP)) {
    if (lane < K)
      for (int j = 0; j < K; ++j) A[lane * ld + j] = gload(gram, go, K, lane, j);
    __syncthreads();
    if (chol_lower(A, K, ld, lane)) {
      const double t = lane < K ? 2.0 * log2(A[lane * ld + lane].x) - log2(gload(gram, go, K, lane, lane).x) : 0.0;
      gapv = -wave_sum(t) / K;
      ginv = inverse_diag(A, wd, K, ld, lane);
    } else {
      st |= XLMIMO_ST_G_NOT_PD;
    }
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
    bool have_q = ok;
    if (!ok && mism) {
      // an indefinite filter Gram is still a valid filter: Q = G~^-1 by Gauss-Jordan
      __syncthreads();
      if (lane < K)
        for (int j = 0; j < K; ++j) A[lane * ld + j] = gload(filter, go, K, lane, j);
      __syncthreads();
      have_q = gauss_jordan_inverse(A, Q, K, ld, lane);
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
    }
    if (have_q && mism) {
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
    if (schemes & XLMIMO_CORR_GAP) {
      if (lane == 0) rates[rbase + s * n_sch + c] = gapv;
      ++c;
    }
  }
  if (status != nullptr && lane == 0) status[blockIdx.x] = st;
}

// ---------------------------------------------------------------------------
// K <= 16 without the mismatched scheme: every factorisation of a drop runs in
// its own 16-lane group with the matrix in registers (lane i holds row i), so a
// drop's ZF, nominal modified-ZF and per-SNR MMSE/CAP factorisations proceed in
// parallel; rows and pivots move by DPP row broadcasts, with no LDS or barrier.
// Matrices with K < 16 are padded with an identity block: the Cholesky factor
// and the inverse's diagonal of the leading K x K block are unchanged, operation
// by operation.  The factorisation's arithmetic is the generic kernel's in the
// same order; the inverse's diagonal sums its squared entries in another order.
//
// Jobs of a drop, in order: [G (ZF)] [G~ (MZF)] then one per SNR when MMSE, CAP
// or MRC is asked for (MRC needs no factorisation and rides on that job).
constexpr int kSmallK = 16;

// Lane `src` of each 16-lane row to the whole row: a DPP row broadcast (a VALU
// move, no LDS round trip, and no initial value: every lane of the row is written).
// src is a constant once the callers' loops unroll.
__device__ __forceinline__ int row_bcast(int v, int src) {
  switch (src) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0x150, 0xF, 0xF, false);
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x151, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x152, 0xF, 0xF, false);
    case 3: return __builtin_amdgcn_mov_dpp(v, 0x153, 0xF, 0xF, false);
    case 4: return __builtin_amdgcn_mov_dpp(v, 0x154, 0xF, 0xF, false);
    case 5: return __builtin_amdgcn_mov_dpp(v, 0x155, 0xF, 0xF, false);
    case 6: return __builtin_amdgcn_mov_dpp(v, 0x156, 0xF, 0xF, false);
    case 7: return __builtin_amdgcn_mov_dpp(v, 0x157, 0xF, 0xF, false);
    case 8: return __builtin_amdgcn_mov_dpp(v, 0x158, 0xF, 0xF, false);
    case 9: return __builtin_amdgcn_mov_dpp(v, 0x159, 0xF, 0xF, false);
    case 10: return __builtin_amdgcn_mov_dpp(v, 0x15A, 0xF, 0xF, false);
    case 11: return __builtin_amdgcn_mov_dpp(v, 0x15B, 0xF, 0xF, false);
    case 12: return __builtin_amdgcn_mov_dpp(v, 0x15C, 0xF, 0xF, false);
    case 13: return __builtin_amdgcn_mov_dpp(v, 0x15D, 0xF, 0xF, false);
    case 14: return __builtin_amdgcn_mov_dpp(v, 0x15E, 0xF, 0xF, false);
    default: return __builtin_amdgcn_mov_dpp(v, 0x15F, 0xF, 0xF, false);
  }
}

__device__ __forceinline__ double bcast16(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)row_bcast((int)(unsigned)u, src);
  const unsigned hi = (unsigned)row_bcast((int)(unsigned)(u >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ cplx shfl16(cplx v, int src) { return {bcast16(v.x, src), bcast16(v.y, src)}; }

// A DPP move of a double within each 16-lane row.
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// One halving step of a reduce-scatter over the row: of the 2H values each lane holds
// (ordered by index, the halves split by index bit MASK), the lane keeps the half its
// own bit MASK selects (the upper half when set) and adds the partner's copy of that
// half.  The partner (DPP control CTRL) agrees with the lane in every index bit above
// MASK, so both hold the same index set, and differs in bit MASK: lane 15 - i (row
// mirror) for bit 3, i ^ 7 (half-row mirror) for bit 2, i ^ 2 and i ^ 1 (quad
// permutations) for bits 1 and 0.
template <int H, int MASK, int CTRL>
__device__ __forceinline__ void halve16(double (&v)[kSmallK], int li) {
  const bool up = li & MASK;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double keep = up ? v[H + j] : v[j];
    const double send = up ? v[j] : v[H + j];
    v[j] = keep + dpp64<CTRL>(send);
  }
}

__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = kSmallK / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kSmallK);
  return v;
}

// Right-looking Cholesky of the padded 16 x 16 matrix whose row `li` is in a[]:
// on return a[c] (c <= li) holds L_{li,c}; diag = L_{li,li}.  ok stays false
// after a non-positive or non-finite pivot (the later arithmetic then runs on
// NaNs harmlessly; the caller discards it).
__device__ __forceinline__ bool chol_rows(cplx (&a)[kSmallK], int li, double& diag) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < kSmallK; ++j) {
    const double djj = bcast16(a[j].x, j);
    ok = ok && (djj > 0.0) && isfinite(djj);
    const double l = sqrt(djj), il = 1.0 / l;
    a[j] = {a[j].x * il, a[j].y * il};
    if (li == j) {
      a[j] = {l, 0.0};
      diag = l;
    }
    // every lane updates; rows above c (li < c) only churn their unused upper triangle, which
    // nothing reads (the inverse below selects L_{li,m} for li > m only), so no lane masks
#pragma unroll
    for (int c = j + 1; c < kSmallK; ++c) {
      const cplx lcj = shfl16(a[j], c);
      const cplx t = cmulc(a[j], lcj);
      a[c] = {a[c].x - t.x, a[c].y - t.y};
    }
  }
  return ok;
}

// [ (L L^H)^-1 ]_{li,li} = sum_i |W_{i,li}|^2 with W = L^-1, built row by row
// in place of L: at step m lane m's row of W is complete up to the scale -1 / L_mm
// (W_mm = 1 / L_mm), the row is broadcast, and every later row i adds
// L_{i,m} W_{m,k} to its running sum for W_{i,k}.  L_{i,m} is read for the last
// time at step m, where slot m of row i starts to accumulate, so one array of 16
// values per lane holds both.  At the end lane i holds -L_ii W_{i,k} for k < i
// and zeros from slot i on; the squared column norms are summed across the rows
// by a reduce-scatter (four halving steps), which leaves column li in lane li.
__device__ __forceinline__ double inv_diag_inplace(cplx (&a)[kSmallK], int li) {
  double guard = 0.0, w = 0.0;   // w: the lane's own 1 / L_{li,li}, kept from step li
#pragma unroll
  for (int m = 0; m < kSmallK; ++m) {
    // a[m] is untouched by the earlier steps; tying it to the previous step's
    // result keeps the compiler from evaluating every step's pivot up front (16
    // live reciprocals and multipliers would push the kernel to one wave per SIMD)
    cplx am = a[m];
    asm volatile("" : "+v"(am.x), "+v"(am.y) : "v"(guard));
    const double w0 = 1.0 / bcast16(am.x, m);             // 1 / L_mm
    if (li == m) w = w0;
    // L_{li,m} for the rows below m, zero elsewhere: adding t * W_{m,k} = 0
    // leaves the other rows unchanged
    const cplx t = li > m ? am : cplx{0.0, 0.0};
    a[m] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k <= m; ++k) {
      // W_{m,k}: lane m holds the unscaled sum, every lane applies -1 / L_mm
      const cplx raw = shfl16(a[k], m);
      const cplx wmk = k == m ? cplx{w0, 0.0} : cplx{raw.x * -w0, raw.y * -w0};
      const cplx u = cmul(t, wmk);
      a[k] = {a[k].x + u.x, a[k].y + u.y};
    }
    guard = a[m].x;   // the step's last update
  }
  const double w2 = w * w;
  double v[kSmallK];
#pragma unroll
  for (int k = 0; k < kSmallK; ++k) v[k] = k == li ? w2 : (a[k].x * a[k].x + a[k].y * a[k].y) * w2;
  halve16<8, 8, 0x140>(v, li);   // row_mirror
  halve16<4, 4, 0x141>(v, li);   // row_half_mirror
  halve16<2, 2, 0x4E>(v, li);    // quad_perm [2, 3, 0, 1]
  halve16<1, 1, 0xB1>(v, li);    // quad_perm [1, 0, 3, 2]
  return v[0];
}

__device__ __forceinline__ void load_row(cplx (&a)[kSmallK], const double* g, int64_t off, int K, int li) {
#pragma unroll
  for (int j = 0; j < kSmallK; ++j)
    a[j] = (li < K && j < K) ? gload(g, off, K, li, j) : cplx{li == j ? 1.0 : 0.0, 0.0};
}

__global__ __launch_bounds__(256) void k_rates_small(const DropK* __restrict__ drops, int n_drops,
                                                      const double* __restrict__ gram,
                                                      const double* __restrict__ filter, int n_snr,
                                                      const double* __restrict__ rho, int64_t total_users,
                                                      int schemes, int n_sch, int jobs, int drops_per_block,
                                                      double* __restrict__ rates, int32_t* __restrict__ status) {
  __shared__ int s_st[64];
  const int group = threadIdx.x / kSmallK, li = threadIdx.x % kSmallK;
  const int slot = group / jobs, job = group % jobs;
  const int64_t d = (int64_t)blockIdx.x * drops_per_block + slot;
  if ((int)threadIdx.x < drops_per_block) s_st[threadIdx.x] = 0;
  __syncthreads();
  const bool zf = schemes & XLMIMO_ZF, mzf = schemes & XLMIMO_MZF, gap = schemes & XLMIMO_CORR_GAP;
  const bool mmse = schemes & XLMIMO_MMSE, cap = schemes & XLMIMO_CAP, mrc = schemes & XLMIMO_MRC;
  // rate column of each scheme: ZF, MMSE, MRC, CAP, MZF, CORR_GAP (the mismatched scheme is not
  // handled here); the factorisation of G serves ZF and the correlation gap
  const int c_mmse = zf, c_mrc = c_mmse + mmse, c_cap = c_mrc + mrc, c_mzf = c_cap + cap, c_gap = c_mzf + mzf;
  const double nan = __builtin_nan("");
  int st = 0;
  if (slot < drops_per_block && d < n_drops) {   // groups past the last slot of the block idle
    const DropK dp = drops[d];
    const int K = dp.k;
    const int64_t go = dp.gram_off;
    const int64_t rbase = d * n_snr * n_sch;
    int kind = job;                        // 0: G, 1: G~, 2 + s: SNR s
    if (!(zf || gap)) ++kind;
    if (!mzf && kind >= 1) ++kind;
    cplx a[kSmallK];
    double diag = 1.0;
    const int s = kind - 2;                 // SNR of an MMSE/CAP/MRC job
    const double* rs = rho + (int64_t)(kind >= 2 ? s : 0) * total_users + dp.user_off;
    const double rk = li < K ? rs[li] : 0.0;
    const bool fact = kind <= 1 || mmse || cap;
    if (kind <= 1) {
      load_row(a, kind == 0 ? gram : filter, go, K, li);
    } else if (fact) {
      // I + D^1/2 G D^1/2, row li
      const double sk = sqrt(rk);
#pragma unroll
      for (int j = 0; j < kSmallK; ++j) {
        if (li < K && j < K) {
          const cplx g = gload(gram, go, K, li, j);
          const double sj = sqrt(rs[j]);
          a[j] = {(li == j ? 1.0 : 0.0) + sk * sj * g.x, sk * sj * g.y};
        } else {
          a[j] = {li == j ? 1.0 : 0.0, 0.0};
        }
      }
    }
    bool ok = true;
    double minv = nan;
    if (fact) {
      ok = chol_rows(a, li, diag);
      minv = inv_diag_inplace(a, li);
    }
    if (kind <= 1) {
      // ZF on the true Gram or nominal modified ZF on the filter Gram, all SNRs
      if (!ok) st |= kind == 0 ? XLMIMO_ST_G_NOT_PD : XLMIMO_ST_FILTER_NOT_PD;
      const double ginv = ok ? minv : nan;
      if (kind == 1 || zf) {
        for (int q = 0; q < n_snr; ++q) {
          const double rq = li < K ? rho[(int64_t)q * total_users + dp.user_off + li] : 0.0;
          const double tot = group_sum(li < K ? log2(1.0 + rq / ginv) : 0.0);
          if (li == 0) rates[rbase + q * n_sch + (kind == 0 ? 0 : c_mzf)] = tot;
        }
      }
      if (kind == 0 && gap) {
        // -(1/K) log2 det R = -(1/K) (2 sum log2 L_kk - sum log2 G_kk), the same for every SNR
        const double t = li < K ? 2.0 * log2(diag) - log2(gload(gram, go, K, li, li).x) : 0.0;
        const double v = ok ? -group_sum(t) / K : nan;
        if (li == 0)
          for (int q = 0; q < n_snr; ++q) rates[rbase + q * n_sch + c_gap] = v;
      }
    } else {
      if (mrc) {
        double v = 0.0;
        if (li < K) {
          const double gkk = gload(gram, go, K, li, li).x;
          double interf = 0.0;
          for (int j = 0; j < K; ++j) {
            if (j == li) continue;
            const cplx g = gload(gram, go, K, li, j);
            interf += rs[j] * (g.x * g.x + g.y * g.y);
          }
          v = log2(1.0 + rk * gkk * gkk / (interf + gkk));
        }
        const double tot = group_sum(v);
        if (li == 0) rates[rbase + s * n_sch + c_mrc] = tot;
      }
      if (fact) {
        const double logd = group_sum(li < K ? log2(diag) : 0.0);
        const double tm = group_sum(li < K ? -log2(minv) : 0.0);
        if (!ok) st |= XLMIMO_ST_MMSE_NOT_PD;
        if (li == 0) {
          if (mmse) rates[rbase + s * n_sch + c_mmse] = ok ? tm : nan;
          if (cap) rates[rbase + s * n_sch + c_cap] = ok ? 2.0 * logd : nan;
        }
      }
    }
    if (st != 0 && li == 0) atomicOr(&s_st[slot], st);   // bitwise OR: the order does not matter
  }
  __syncthreads();
  if (status != nullptr && (int)threadIdx.x < drops_per_block) {
    const int64_t dd = (int64_t)blockIdx.x * drops_per_block + threadIdx.x;
    if (dd < n_drops) status[dd] = s_st[threadIdx.x];
  }
}

// ---------------------------------------------------------------------------
// K > XLMIMO_MAX_USERS: one 512-thread workgroup per drop, each factorisation's
// matrix in a global workspace as a column-major lower triangle (element
// (i, j), i >= j, at M[j K + i]).  Blocked right-looking Cholesky (chol_global):
// every thread updates whole rows, so a wave's accesses to one column are
// contiguous.  W = L^-1 is then formed row by row, W_ik = -(1/L_ii) sum_{k <= t < i} L_it W_tk,
// with W_ik (k < i) kept in the unused upper triangle at M[i K + k], so
// [M^-1]_kk = sum_i |W_ik|^2.  The SINRs, NaN and status conventions and the
// column order are those of k_rates; sums over users run in a fixed order.
constexpr int kLargeThreads = 512;

// Sum over the workgroup in a fixed order (per-thread sums, wave butterfly,
// then the waves in order); every thread gets the total.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kLargeThreads / 64; ++w) t += red[w];
  return t;
}

// Blocked right-looking Cholesky in panels of kPanel columns.  A panel is
// factorised one column at a time (each finished column is staged in LDS and
// updates only the panel's later columns); then the trailing triangle takes the
// panel's rank-kPanel update in one pass: thread i holds L_i,panel in registers
// and walks the columns c <= i, two at a time, reading L_c,panel from LDS (a
// broadcast) and M[c K + i] once.  The trailing triangle is read and written
// once per panel instead of once per column.
constexpr int kPanel = 8;

__device__ bool chol_global(cplx* M, int K, cplx* s_pan) {
  const int tid = threadIdx.x;
  for (int j0 = 0; j0 < K; j0 += kPanel) {
    const int jp = min(kPanel, K - j0);
    for (int p = 0; p < jp; ++p) {
      const int j = j0 + p;
      __syncthreads();                                   // the previous step's updates are visible
      const double djj = M[(int64_t)j * K + j].x;
      if (!(djj > 0.0) || !isfinite(djj)) return false;  // uniform: every thread read the same pivot
      const double l = sqrt(djj), il = 1.0 / l;
      for (int i = j + 1 + tid; i < K; i += kLargeThreads) {
        const cplx v = M[(int64_t)j * K + i];
        const cplx w = {v.x * il, v.y * il};
        M[(int64_t)j * K + i] = w;
        s_pan[p * K + i] = w;
      }
      __syncthreads();
      if (tid == 0) M[(int64_t)j * K + j] = {l, 0.0};
      // the panel's later columns c in (j, j0 + jp), rows i >= c
      for (int i = j + 1 + tid; i < K; i += kLargeThreads) {
        const cplx lij = s_pan[p * K + i];
        const int c1 = min(i, j0 + jp - 1);
        for (int c = j + 1; c <= c1; ++c) {
          const cplx t = cmulc(lij, s_pan[p * K + c]);
          const cplx v = M[(int64_t)c * K + i];
          M[(int64_t)c * K + i] = {v.x - t.x, v.y - t.y};
        }
      }
    }
    __syncthreads();
    // trailing update (a panel with a trailing part is always full: jp == kPanel)
    const int c0 = j0 + jp;
    for (int i = c0 + tid; i < K; i += kLargeThreads) {
      cplx li[kPanel];
#pragma unroll
      for (int p = 0; p < kPanel; ++p) li[p] = s_pan[p * K + i];
      int c = c0;
      for (; c < i; c += 2) {
        cplx a0 = M[(int64_t)c * K + i], a1 = M[(int64_t)(c + 1) * K + i];
#pragma unroll
        for (int p = 0; p < kPanel; ++p) {
          const cplx t0 = cmulc(li[p], s_pan[p * K + c]);
          const cplx t1 = cmulc(li[p], s_pan[p * K + c + 1]);
          a0.x -= t0.x;
          a0.y -= t0.y;
          a1.x -= t1.x;
          a1.y -= t1.y;
        }
        M[(int64_t)c * K + i] = a0;
        M[(int64_t)(c + 1) * K + i] = a1;
      }
      if (c == i) {
        cplx a0 = M[(int64_t)c * K + i];
#pragma unroll
        for (int p = 0; p < kPanel; ++p) {
          const cplx t0 = cmulc(li[p], s_pan[p * K + c]);
          a0.x -= t0.x;
          a0.y -= t0.y;
        }
        M[(int64_t)c * K + i] = a0;
      }
    }
  }
  __syncthreads();
  return true;
}

// Diagonal of (L L^H)^-1 for the factor L in M, into s_inv[0, K).  W = L^-1 is
// formed kPanel rows at a time: those rows of L are staged in LDS (s_rows,
// kPanel x K), and thread k, for its columns k, sums the earlier rows'
// contributions sum_{t < i0} L_it W_tk for all kPanel rows from one read of
// each W_tk, then runs the rows' own recurrence in registers.  W_ik (k < i) is
// kept in the unused upper triangle at M[i K + k].
__device__ void inv_diag_global(cplx* M, int K, cplx* s_rows, double* s_inv) {
  const int tid = threadIdx.x;
  for (int k = tid; k < K; k += kLargeThreads) {
    const double w = 1.0 / M[(int64_t)k * K + k].x;
    s_inv[k] = w * w;
  }
  for (int i0 = 0; i0 < K; i0 += kPanel) {
    const int nr = min(kPanel, K - i0);
    __syncthreads();                                   // earlier rows of W are written, s_rows is free
    for (int r = 0; r < nr; ++r)
      for (int t = tid; t <= i0 + r; t += kLargeThreads) s_rows[r * K + t] = M[(int64_t)t * K + i0 + r];   // L_{i0+r,t}
    __syncthreads();
    for (int k = tid; k < i0 + nr; k += kLargeThreads) {
      const double wkk = 1.0 / M[(int64_t)k * K + k].x;
      cplx acc[kPanel];
#pragma unroll
      for (int r = 0; r < kPanel; ++r) acc[r] = {0.0, 0.0};
      if (k < i0) {
        // earlier rows: t = k (W_kk), then t in (k, i0) from the wave's first column on, so that a
        // wave reads one row of W contiguously; terms with t <= k are multiplied by zero
#pragma unroll
        for (int r = 0; r < kPanel; ++r)
          if (r < nr) acc[r] = {s_rows[r * K + k].x * wkk, s_rows[r * K + k].y * wkk};
        const int t0 = (k & ~63) + 1;
        // four loads of W in flight per step (the sums keep their order over t)
        int t = t0;
        for (; t + 4 <= i0; t += 4) {
          cplx m[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) m[u] = M[(int64_t)(t + u) * K + k];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const cplx w = t + u > k ? m[u] : cplx{0.0, 0.0};
#pragma unroll
            for (int r = 0; r < kPanel; ++r) {
              if (r < nr) {
                const cplx p = cmul(s_rows[r * K + t + u], w);
                acc[r].x += p.x;
                acc[r].y += p.y;
              }
            }
          }
        }
        for (; t < i0; ++t) {
          const cplx m = M[(int64_t)t * K + k];
          const cplx w = t > k ? m : cplx{0.0, 0.0};
#pragma unroll
          for (int r = 0; r < kPanel; ++r) {
            if (r < nr) {
              const cplx p = cmul(s_rows[r * K + t], w);
              acc[r].x += p.x;
              acc[r].y += p.y;
            }
          }
        }
      }
      // this block's rows in order: W_ik = -(1/L_ii)(acc + sum_{t in [max(k, i0), i)} L_it W_tk)
      cplx wb[kPanel];
#pragma unroll
      for (int r = 0; r < kPanel; ++r) {
        const int i = i0 + r;
        wb[r] = {0.0, 0.0};
        if (r >= nr || i < k) continue;
        if (i == k) {
          wb[r] = {wkk, 0.0};
          continue;
        }
        cplx a = acc[r];
#pragma unroll
        for (int q = 0; q < kPanel; ++q) {
          if (q < r && i0 + q >= k) {
            const cplx p = cmul(s_rows[r * K + i0 + q], wb[q]);
            a.x += p.x;
            a.y += p.y;
          }
        }
        const double ili = 1.0 / s_rows[r * K + i].x;
        wb[r] = {-a.x * ili, -a.y * ili};
        M[(int64_t)i * K + k] = wb[r];
        s_inv[k] += wb[r].x * wb[r].x + wb[r].y * wb[r].y;
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kLargeThreads) void k_rates_large(const DropK* __restrict__ drops,
                                                               const double* __restrict__ gram, int n_snr,
                                                               const double* __restrict__ rho, int64_t total_users,
                                                               int schemes, int n_sch, double* __restrict__ work,
                                                               double* __restrict__ rates,
                                                               int32_t* __restrict__ status) {
  __shared__ cplx s_vec[kPanel * XLMIMO_MAX_USERS_EXACT];   // Cholesky panel; row of L in the inverse
  __shared__ double s_inv[XLMIMO_MAX_USERS_EXACT], s_ginv[XLMIMO_MAX_USERS_EXACT];
  __shared__ double s_red[kLargeThreads / 64];
  const int tid = threadIdx.x;
  const DropK dp = drops[blockIdx.x];
  const int K = dp.k;
  const int64_t KK = (int64_t)K * K;
  const cplx* G = reinterpret_cast<const cplx*>(gram) + dp.gram_off;
  cplx* M = reinterpret_cast<cplx*>(work) + dp.gram_off;
  const double nan = __builtin_nan("");
  int st = 0;

  // G itself: ZF's [G^-1]_kk and the correlation gap -(1/K) log2 det R
  double gap = nan;
  bool g_ok = false;
  if (schemes & (XLMIMO_ZF | XLMIMO_CORR_GAP)) {
    // M_ic = G_ic = conj(G_ci): row c of the row-major Gram is column c of M
    for (int64_t e = tid; e < KK; e += kLargeThreads) {
      const int c = (int)(e / K), i = (int)(e - (int64_t)c * K);
      if (i >= c) M[e] = {G[e].x, -G[e].y};
    }
    g_ok = chol_global(M, K, s_vec);
    if (g_ok) {
      double t = 0.0;
      for (int k = tid; k < K; k += kLargeThreads)
        t += 2.0 * log2(M[(int64_t)k * K + k].x) - log2(G[(int64_t)k * K + k].x);
      gap = -block_sum(t, s_red) / K;
      if (schemes & XLMIMO_ZF) {
        inv_diag_global(M, K, s_vec, s_inv);
        for (int k = tid; k < K; k += kLargeThreads) s_ginv[k] = s_inv[k];
      }
    } else {
      st |= XLMIMO_ST_G_NOT_PD;
    }
  }

  const int64_t rbase = (int64_t)blockIdx.x * n_snr * n_sch;
  for (int s = 0; s < n_snr; ++s) {
    const double* rs = rho + (int64_t)s * total_users + dp.user_off;
    int col = 0;
    if (schemes & XLMIMO_ZF) {
      double v = 0.0;
      for (int k = tid; k < K; k += kLargeThreads) v += g_ok ? log2(1.0 + rs[k] / s_ginv[k]) : nan;
      const double tot = block_sum(v, s_red);
      if (tid == 0) rates[rbase + s * n_sch + col] = tot;
      ++col;
    }
    double cap = nan;
    if (schemes & (XLMIMO_MMSE | XLMIMO_CAP)) {
      // I + D^1/2 G D^1/2, lower triangle
      for (int64_t e = tid; e < KK; e += kLargeThreads) {
        const int c = (int)(e / K), i = (int)(e - (int64_t)c * K);
        if (i >= c) {
          const double f = sqrt(rs[i]) * sqrt(rs[c]);
          M[e] = {(i == c ? 1.0 : 0.0) + f * G[e].x, -f * G[e].y};
        }
      }
      double mmse = nan;
      if (chol_global(M, K, s_vec)) {
        double t = 0.0;
        for (int k = tid; k < K; k += kLargeThreads) t += log2(M[(int64_t)k * K + k].x);
        cap = 2.0 * block_sum(t, s_red);
        if (schemes & XLMIMO_MMSE) {
          inv_diag_global(M, K, s_vec, s_inv);
          double u = 0.0;
          for (int k = tid; k < K; k += kLargeThreads) u -= log2(s_inv[k]);   // log2(1 + SINR) = -log2 [M^-1]_kk
          mmse = block_sum(u, s_red);
        }
      } else {
        st |= XLMIMO_ST_MMSE_NOT_PD;
      }
      if (schemes & XLMIMO_MMSE) {
        if (tid == 0) rates[rbase + s * n_sch + col] = mmse;
        ++col;
      }
    }
    if (schemes & XLMIMO_MRC) {
      double v = 0.0;
      for (int k = tid; k < K; k += kLargeThreads) {
        const double gkk = G[(int64_t)k * K + k].x;
        double interf = 0.0;
        for (int j = 0; j < K; ++j) {
          if (j == k) continue;
          const cplx g = G[(int64_t)j * K + k];   // |G_kj| = |G_jk|, contiguous over k
          interf += rs[j] * (g.x * g.x + g.y * g.y);
        }
        v += log2(1.0 + rs[k] * gkk * gkk / (interf + gkk));
      }
      const double tot = block_sum(v, s_red);
      if (tid == 0) rates[rbase + s * n_sch + col] = tot;
      ++col;
    }
    if (schemes & XLMIMO_CAP) {
      if (tid == 0) rates[rbase + s * n_sch + col] = cap;
      ++col;
    }
    if (schemes & XLMIMO_CORR_GAP) {
      if (tid == 0) rates[rbase + s * n_sch + col] = gap;
      ++col;
    }
  }
  if (status != nullptr && tid == 0) status[blockIdx.x] = st;
}

// ---------------------------------------------------------------------------
// Cholesky factors for tracking.  The factored matrix is G (rho == nullptr) or
// I + D^1/2 G D^1/2 with D = diag(rho) for one SNR; its factor L is kept in
// LAPACK column-major order (element (i, j), i >= j, at [j K + i] of the drop's
// K x K block at its Gram offset), the strict upper triangle zero.

__device__ double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kLargeThreads / 64; ++w) t = fmax(t, red[w]);
  return t;
}

// log2 det of the factored matrix, 2 sum log2 L_kk (fixed order; every thread gets it)
__device__ double factor_log2det(const cplx* M, int K, double* red) {
  double t = 0.0;
  for (int k = threadIdx.x; k < K; k += kLargeThreads) t += log2(M[(int64_t)k * K + k].x);
  return 2.0 * block_sum(t, red);
}

__global__ __launch_bounds__(kLargeThreads) void k_cholesky(const DropK* __restrict__ drops,
                                                            const double* __restrict__ gram,
                                                            const double* __restrict__ rho,
                                                            double* __restrict__ factor,
                                                            double* __restrict__ logdet,
                                                            int32_t* __restrict__ status) {
  __shared__ cplx s_pan[kPanel * XLMIMO_MAX_USERS_EXACT];
  __shared__ double s_red[kLargeThreads / 64];
  const DropK dp = drops[blockIdx.x];
  const int K = dp.k;
  const int64_t KK = (int64_t)K * K;
  const cplx* G = reinterpret_cast<const cplx*>(gram) + dp.gram_off;
  cplx* M = reinterpret_cast<cplx*>(factor) + dp.gram_off;
  const double* rs = rho != nullptr ? rho + dp.user_off : nullptr;
  // element (i, c) = conj(G_ci): row c of the row-major Gram is column c of M
  for (int64_t e = threadIdx.x; e < KK; e += kLargeThreads) {
    const int c = (int)(e / K), i = (int)(e - (int64_t)c * K);
    if (i < c) {
      M[e] = {0.0, 0.0};
    } else if (rs != nullptr) {
      const double f = sqrt(rs[i]) * sqrt(rs[c]);
      M[e] = {(i == c ? 1.0 : 0.0) + f * G[e].x, -f * G[e].y};
    } else {
      M[e] = {G[e].x, -G[e].y};
    }
  }
  const bool ok = chol_global(M, K, s_pan);
  double ld = __builtin_nan("");
  if (ok) ld = factor_log2det(M, K, s_red);
  if (threadIdx.x == 0) {
    if (logdet != nullptr) logdet[blockIdx.x] = ld;
    if (status != nullptr) status[blockIdx.x] = ok ? 0 : (rho != nullptr ? XLMIMO_ST_MMSE_NOT_PD : XLMIMO_ST_G_NOT_PD);
  }
}

// Moved users of one drop per workgroup (drop mdrop[b], users mloc[moff[b] .. moff[b + 1]), ascending).
// Row and column m of the factored matrix A changed: Delta = u e_m^H + e_m u^H with u the new column m
// minus the old one (the old row from L L^H, u_m halved), = v1 v1^H - v2 v2^H for
// v1,2 = (u / s +- s e_m) / sqrt 2.  One pass over the columns applies, at column k, the rotation
// of the update with v1 and then the hyperbolic rotation of the downdate with v2 to column k and
// to the vectors' later entries.  A downdate pivot <= 0 (A no longer positive definite) stops the
// drop with the status bit set and log2 det NaN.
__global__ __launch_bounds__(kLargeThreads) void k_chol_update(const DropK* __restrict__ drops,
                                                               const int32_t* __restrict__ mdrop,
                                                               const int32_t* __restrict__ moff,
                                                               const int32_t* __restrict__ mloc,
                                                               const double* __restrict__ gram,
                                                               const double* __restrict__ rho,
                                                               double* __restrict__ factor,
                                                               double* __restrict__ logdet,
                                                               int32_t* __restrict__ status) {
  __shared__ cplx s_l[XLMIMO_MAX_USERS_EXACT], s_v1[XLMIMO_MAX_USERS_EXACT], s_v2[XLMIMO_MAX_USERS_EXACT];
  __shared__ double s_red[kLargeThreads / 64];
  const int tid = threadIdx.x;
  const int d = mdrop[blockIdx.x];
  const DropK dp = drops[d];
  const int K = dp.k;
  const cplx* G = reinterpret_cast<const cplx*>(gram) + dp.gram_off;
  cplx* M = reinterpret_cast<cplx*>(factor) + dp.gram_off;
  const double* rs = rho != nullptr ? rho + dp.user_off : nullptr;
  bool ok = true;
  for (int q = moff[blockIdx.x]; q < moff[blockIdx.x + 1] && ok; ++q) {
    const int m = mloc[q];
    __syncthreads();                                        // the previous user's pass is complete
    for (int k = tid; k <= m; k += kLargeThreads) s_l[k] = M[(int64_t)k * K + m];   // row m of L
    __syncthreads();
    double umax = 0.0;
    for (int j = tid; j < K; j += kLargeThreads) {
      cplx a = {0.0, 0.0};                                  // old (L L^H)_mj = sum_k L_mk conj(L_jk)
      const int kmax = min(m, j);
      for (int k = 0; k <= kmax; ++k) {
        const cplx t = cmulc(s_l[k], M[(int64_t)k * K + j]);
        a.x += t.x;
        a.y += t.y;
      }
      const cplx g = G[(int64_t)m * K + j];                 // new G_mj
      cplx an = g;
      if (rs != nullptr) {
        const double f = sqrt(rs[m]) * sqrt(rs[j]);
        an = {(j == m ? 1.0 : 0.0) + f * g.x, f * g.y};
      }
      const cplx dl = {an.x - a.x, an.y - a.y};             // Delta_mj
      const cplx u = j == m ? cplx{0.5 * dl.x, 0.0} : cplx{dl.x, -dl.y};   // Delta_jm, u_m halved
      s_v1[j] = u;
      umax = fmax(umax, fmax(fabs(u.x), fabs(u.y)));
    }
    umax = block_max(umax, s_red);
    if (!isfinite(umax)) {
      ok = false;
      break;
    }
    if (!(umax > 0.0)) continue;                            // row unchanged (uniform)
    const double sc = sqrt(umax), isc = 1.0 / sc, h = 0.70710678118654752440;
    for (int j = tid; j < K; j += kLargeThreads) {
      const cplx u = s_v1[j];
      const double em = j == m ? sc : 0.0;
      s_v1[j] = {(u.x * isc + em) * h, u.y * isc * h};
      s_v2[j] = {(u.x * isc - em) * h, u.y * isc * h};
    }
    for (int k = 0; k < K; ++k) {
      __syncthreads();                                      // column k - 1 and the vectors are written
      const double lkk = M[(int64_t)k * K + k].x;
      const cplx x1 = s_v1[k], x2 = s_v2[k];
      const double ra = sqrt(fma(lkk, lkk, x1.x * x1.x + x1.y * x1.y));
      const double rb2 = ra * ra - (x2.x * x2.x + x2.y * x2.y);
      if (!(rb2 > 0.0) || !isfinite(rb2)) {                 // uniform: every thread read the same values
        ok = false;
        break;
      }
      const double rb = sqrt(rb2), ia = 1.0 / ra, ib = 1.0 / rb;
      __syncthreads();                                      // every thread has read L_kk, x1_k, x2_k
      for (int i = k + 1 + tid; i < K; i += kLargeThreads) {
        const cplx li = M[(int64_t)k * K + i];
        cplx y1 = s_v1[i], y2 = s_v2[i];
        const cplx c1 = cconjmul(x1, y1), c2 = cmul(x1, li);
        const cplx l1 = {(lkk * li.x + c1.x) * ia, (lkk * li.y + c1.y) * ia};
        y1 = {(lkk * y1.x - c2.x) * ia, (lkk * y1.y - c2.y) * ia};
        const cplx c3 = cconjmul(x2, y2), c4 = cmul(x2, l1);
        M[(int64_t)k * K + i] = {(ra * l1.x - c3.x) * ib, (ra * l1.y - c3.y) * ib};
        y2 = {(ra * y2.x - c4.x) * ib, (ra * y2.y - c4.y) * ib};
        s_v1[i] = y1;
        s_v2[i] = y2;
      }
      if (tid == 0) M[(int64_t)k * K + k] = {rb, 0.0};
    }
  }
  __syncthreads();
  double ld = __builtin_nan("");
  if (ok) ld = factor_log2det(M, K, s_red);
  if (tid == 0) {
    if (logdet != nullptr) logdet[d] = ld;
    if (status != nullptr) status[d] = ok ? 0 : (rho != nullptr ? XLMIMO_ST_MMSE_NOT_PD : XLMIMO_ST_G_NOT_PD);
  }
}

hipError_t launch_cholesky(const DropK* d_drops, int n_drops, const double* d_gram, const double* d_rho,
                           double* d_factor, double* d_logdet, int32_t* d_status, hipStream_t s) {
  if (n_drops == 0) return hipSuccess;
  k_cholesky<<<n_drops, kLargeThreads, 0, s>>>(d_drops, d_gram, d_rho, d_factor, d_logdet, d_status);
  return hipGetLastError();
}

hipError_t launch_chol_update(const DropK* d_drops, int n_mdrops, const int32_t* d_mdrop, const int32_t* d_moff,
                              const int32_t* d_mloc, const double* d_gram, const double* d_rho, double* d_factor,
                              double* d_logdet, int32_t* d_status, hipStream_t s) {
  if (n_mdrops == 0) return hipSuccess;
  k_chol_update<<<n_mdrops, kLargeThreads, 0, s>>>(d_drops, d_mdrop, d_moff, d_mloc, d_gram, d_rho, d_factor,
                                                  d_logdet, d_status);
  return hipGetLastError();
}

hipError_t launch_rates(const DropK* d_drops, int n_drops, int k_max, const double* d_gram, const double* d_filter,
                        int n_snr, const double* d_rho, int64_t total_users, int schemes, double* d_rates,
                        int32_t* d_status, hipStream_t s, double* d_work) {
  if (n_drops == 0) return hipSuccess;
  int n_sch = __builtin_popcount(schemes);
  if (k_max > XLMIMO_MAX_USERS) {
    if (d_work == nullptr || (schemes & (XLMIMO_MZF | XLMIMO_MZF_MISM))) return hipErrorInvalidValue;
    k_rates_large<<<n_drops, kLargeThreads, 0, s>>>(d_drops, d_gram, n_snr, d_rho, total_users, schemes, n_sch,
                                                    d_work, d_rates, d_status);
    return hipGetLastError();
  }
  const int ld = k_max + 1;
  const bool mism = schemes & XLMIMO_MZF_MISM;
  const int jobs = ((schemes & (XLMIMO_ZF | XLMIMO_CORR_GAP)) ? 1 : 0) + ((schemes & XLMIMO_MZF) ? 1 : 0) +
                   ((schemes & (XLMIMO_MMSE | XLMIMO_CAP | XLMIMO_MRC)) ? n_snr : 0);
  if (k_max <= kSmallK && !mism && jobs >= 1 && jobs * kSmallK <= 256) {
    // several drops per wave when a drop needs fewer than four factorisations
    const int per = jobs >= 4 ? 1 : 4 / jobs;
    const int threads = ((per * jobs * kSmallK + 63) / 64) * 64;
    const int blocks = (int)((n_drops + per - 1) / per);
    k_rates_small<<<blocks, threads, 0, s>>>(d_drops, n_drops, d_gram, d_filter, n_snr, d_rho, total_users, schemes,
                                             n_sch, jobs, per, d_rates, d_status);
    return hipGetLastError();
  }
  const size_t lds = (size_t)(mism ? 2 : 1) * k_max * ld * sizeof(cplx) + 64 * sizeof(double);
  k_rates<<<n_drops, 64, lds, s>>>(d_drops, d_gram, d_filter, n_snr, d_rho, total_users, schemes, n_sch, d_rates,
                                    d_status, ld);
  return hipGetLastError();
}

}  // namespace xl
