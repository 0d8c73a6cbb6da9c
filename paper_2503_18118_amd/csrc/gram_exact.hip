// Exact multiuser Gram G = H^H H with H generated on the fly (never stored).
//
// Sec. III defines P_i = P ||h_i||^2 and rho_ij = h_i^H h_j / (||h_i|| ||h_j||);
// Sec. V-B names these length-N inner products as the cost the paper wants to
// remove.  Here they are computed exactly, for a batch of drops of uneven N, K.
//
// Work decomposition
//   A work item is a contiguous element range of one drop.  A persistent grid
//   of 256-thread workgroups pops items from an atomic queue (items are sorted
//   by decreasing cost on the host, so the queue is a longest-first schedule).
//   Inside an item, each round covers 16 elements: wave w takes elements
//   4w..4w+3, lane l evaluates user 16b + (l % 16) at element l / 16 for every
//   16-user block b.  Each lane therefore holds one row of the 4 x 16 MFMA
//   operand "h_re" and "h_im" of every block.
//
// Contraction on the matrix cores (16x16x4 MFMA, A and B from the same lanes):
//   Re G[bi,bj] += sum re_i re_j + im_i im_j      for bi <= bj   (2 MFMA)
//   X[bi,bj]    += sum re_i im_j                  for all bi, bj (1 MFMA)
//   Im G_ij = X_ij - X_ji                          (applied in the finalize pass)
//   i.e. 3 MFMA per 4 elements for K <= 16.
//
// Precision
//   FP32C: distance and phase reduction in FP64 (device_math.h), sin/cos and
//   amplitude in FP32, FP32 MFMA partial sums flushed to FP64 every
//   kFlushRounds rounds (256 elements per wave), FP64 across waves and items.
//   FP64: every step in FP64, FP64 MFMA accumulation.
//   Amplitude constants are applied in FP64 at the end: FREESPACE lanes carry
//   1/r (scale (lambda/4pi)^2), PNUSW lanes carry r^{-3/2} (scale beta0 sqrt(x_i x_j)).
//
// Determinism: every sum has a fixed order (waves in order through LDS, items
// of a drop in chunk order in the finalize pass), so results are bitwise
// repeatable regardless of which workgroup ran which item.
#include "device_math.h"
#include "internal.h"
#include "xlmimo.h"

namespace xl {

struct UserLane {
  double xp2;   // squared distance from the array line (ULA) or plane (UPA)
  double uy, uz;
  bool active;
};

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef floatx4 acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<double> {
  typedef doublex4 acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T>
__device__ __forceinline__ void channel_entry(const ArrayK& arr, double ey, double ez, const UserLane& u, bool valid,
                                              T& re, T& im) {
  const double dy = u.uy - ey;
  double r2 = fma(dy, dy, u.xp2);
  if (arr.geom == XLMIMO_UPA) {
    const double dz = u.uz - ez;
    r2 = fma(dz, dz, r2);
  }
  const double y = (sizeof(T) == 4) ? rsqrt_nr1(r2) : rsqrt_nr2(r2);  // 1 / r
  double t;
  int q;
  reduce_quarter((r2 * y) * arr.inv_lambda, t, q);
  T s, c;
  sincos_rev((T)t, s, c);
  T a = (T)y;
  if (arr.amp == XLMIMO_AMP_PNUSW) {
    if constexpr (sizeof(T) == 4) a = a * __builtin_amdgcn_sqrtf(a);
    else a = a * sqrt(a);
  }
  rotate_conj(a, s, c, q, re, im);
  if (!(valid && u.active)) {
    re = (T)0;
    im = (T)0;
  }
}

template <int NB, typename T>
__device__ void process_item(const ArrayK& arr, const DropK& dp, const ItemK& it, const double* __restrict__ pos,
                             double* __restrict__ part_out, double* s_red) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int NRE = NB * (NB + 1) / 2;
  constexpr int NX = NB * NB;
  constexpr int NV = (NRE + NX) * 4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;

  UserLane u[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int k = 16 * b + (lane & 15);
    u[b].active = k < dp.k;
    double x = 1.0, y = 0.0, z = 0.0;
    if (u[b].active) {
      const double* p = pos + (dp.user_off + k) * 3;
      x = p[0];
      y = p[1];
      z = p[2];
    }
    u[b].xp2 = (arr.geom == XLMIMO_ULA) ? fma(x, x, z * z) : x * x;
    u[b].uy = y;
    u[b].uz = z;
  }

  acc_t are[NRE], ax[NX];
#pragma unroll
  for (int i = 0; i < NRE; ++i) are[i] = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < NX; ++i) ax[i] = acc_t{0, 0, 0, 0};
  double carry[sizeof(T) == 4 ? NV : 1];
#pragma unroll
  for (int i = 0; i < (sizeof(T) == 4 ? NV : 1); ++i) carry[i] = 0.0;

  const int n_rounds = (it.e_end - it.e_begin + 15) >> 4;
  int e = it.e_begin + 4 * wave + (lane >> 4);
  const int ny = (arr.geom == XLMIMO_ULA) ? dp.n_elems : arr.n_y;
  const double cy = 0.5 * (double)(ny - 1) * arr.spacing;
  const double cz = 0.5 * (double)(arr.n_z - 1) * arr.spacing;
  int ea = 0, eb = 0;
  if (arr.geom == XLMIMO_UPA) {
    ea = e / arr.n_z;
    eb = e - ea * arr.n_z;
  }

  for (int r = 0; r < n_rounds; ++r) {
    const bool valid = e < it.e_end;
    double ey, ez = 0.0;
    if (arr.geom == XLMIMO_ULA) {
      ey = fma((double)e, arr.spacing, -cy);
    } else {
      ey = fma((double)ea, arr.spacing, -cy);
      ez = fma((double)eb, arr.spacing, -cz);
    }
    T hre[NB], him[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) channel_entry<T>(arr, ey, ez, u[b], valid, hre[b], him[b]);
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
      for (int bj = bi; bj < NB; ++bj) {
        const int t = tri_index(bi, bj, NB);
        are[t] = Mfma<T>::run(hre[bi], hre[bj], are[t]);
        are[t] = Mfma<T>::run(him[bi], him[bj], are[t]);
      }
    }
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
      for (int bj = 0; bj < NB; ++bj) ax[bi * NB + bj] = Mfma<T>::run(hre[bi], him[bj], ax[bi * NB + bj]);
    }
    e += 16;
    if (arr.geom == XLMIMO_UPA) {
      eb += 16;
      while (eb >= arr.n_z) {
        eb -= arr.n_z;
        ++ea;
      }
    }
    if constexpr (sizeof(T) == 4) {
      if (((r + 1) % kFlushRounds) == 0) {
#pragma unroll
        for (int i = 0; i < NRE; ++i) {
#pragma unroll
          for (int c = 0; c < 4; ++c) carry[i * 4 + c] += (double)are[i][c];
          are[i] = acc_t{0, 0, 0, 0};
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
          for (int c = 0; c < 4; ++c) carry[(NRE + i) * 4 + c] += (double)ax[i][c];
          ax[i] = acc_t{0, 0, 0, 0};
        }
      }
    }
  }

  double fin[NV];
#pragma unroll
  for (int i = 0; i < NRE; ++i) {
#pragma unroll
    for (int c = 0; c < 4; ++c) fin[i * 4 + c] = (double)are[i][c] + (sizeof(T) == 4 ? carry[i * 4 + c] : 0.0);
  }
#pragma unroll
  for (int i = 0; i < NX; ++i) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
      fin[(NRE + i) * 4 + c] = (double)ax[i][c] + (sizeof(T) == 4 ? carry[(NRE + i) * 4 + c] : 0.0);
  }

  // Fixed-order reduction over the 4 waves through LDS.
  for (int w = 0; w < kGramThreads / 64; ++w) {
    if (wave == w) {
#pragma unroll
      for (int v = 0; v < NV; ++v) s_red[v * 64 + lane] = (w == 0) ? fin[v] : s_red[v * 64 + lane] + fin[v];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < NV * 64; i += kGramThreads) part_out[i] = s_red[i];
  __syncthreads();
}

template <int NBMAX, typename T>
__global__ __launch_bounds__(kGramThreads) void k_gram_exact(ArrayK arr, const DropK* __restrict__ drops,
                                                               const double* __restrict__ pos,
                                                               const ItemK* __restrict__ items, int n_items,
                                                               int* __restrict__ counter,
                                                               double* __restrict__ partials) {
  __shared__ double s_red[partial_values(NBMAX) * 64];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = s_item;
    __syncthreads();
    if (idx >= n_items) break;  // uniform over the workgroup: every wave leaves together
    const ItemK it = items[idx];
    const DropK dp = drops[it.drop];
    double* out = partials + dp.part_off + it.chunk * (int64_t)(partial_values(dp.nb) * 64);
    switch (dp.nb) {
      case 1: process_item<1, T>(arr, dp, it, pos, out, s_red); break;
      case 2: if constexpr (NBMAX >= 2) process_item<2, T>(arr, dp, it, pos, out, s_red); break;
      case 3: if constexpr (NBMAX >= 3) process_item<3, T>(arr, dp, it, pos, out, s_red); break;
      case 4: if constexpr (NBMAX >= 4) process_item<4, T>(arr, dp, it, pos, out, s_red); break;
      default: break;
    }
  }
}

__global__ void k_reset_counter(int* counter) {
  if (threadIdx.x == 0) *counter = 0;
}

// Position of C[row][col] of a 16x16 MFMA accumulator in the (value, lane) image.
template <typename T>
__device__ __forceinline__ int acc_slot(int blk, int row, int col) {
  if constexpr (sizeof(T) == 4) {
    // f32 16x16x4: lane l, register r hold C[4 (l / 16) + r][l % 16]
    return (blk * 4 + (row & 3)) * 64 + col + 16 * (row >> 2);
  } else {
    // f64 16x16x4: lane l, register r hold C[4 r + l / 16][l % 16]
    return (blk * 4 + (row >> 2)) * 64 + col + 16 * (row & 3);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gram_finalize(ArrayK arr, const DropK* __restrict__ drops,
                                                       const double* __restrict__ pos,
                                                       const double* __restrict__ partials,
                                                       double* __restrict__ gram) {
  const DropK dp = drops[blockIdx.x];
  const int K = dp.k, NB = dp.nb;
  const int NRE = NB * (NB + 1) / 2;
  const int64_t PV = partial_values(NB) * 64;
  const double* base = partials + dp.part_off;
  for (int idx = threadIdx.x; idx < K * K; idx += blockDim.x) {
    const int i = idx / K, j = idx - (idx / K) * K;
    const int p = i < j ? i : j, q = i < j ? j : i;  // canonical p <= q
    const int bp = p >> 4, pp = p & 15, bq = q >> 4, qq = q & 15;
    const int s_re = acc_slot<T>(tri_index(bp, bq, NB), pp, qq);
    const int s_xpq = acc_slot<T>(NRE + bp * NB + bq, pp, qq);
    const int s_xqp = acc_slot<T>(NRE + bq * NB + bp, qq, pp);
    double re = 0.0, xpq = 0.0, xqp = 0.0;
    for (int c = 0; c < dp.n_items; ++c) {
      const double* pc = base + c * PV;
      re += pc[s_re];
      xpq += pc[s_xpq];
      xqp += pc[s_xqp];
    }
    double im = (p == q) ? 0.0 : xpq - xqp;
    double scale;
    if (arr.amp == XLMIMO_AMP_FREESPACE) {
      const double c0 = arr.lambda / (4.0 * 3.14159265358979323846264338327950288);
      scale = c0 * c0;
    } else {
      const double* up = pos + (dp.user_off + p) * 3;
      const double* uq = pos + (dp.user_off + q) * 3;
      const double xp = (arr.geom == XLMIMO_ULA) ? sqrt(fma(up[0], up[0], up[2] * up[2])) : fabs(up[0]);
      const double xq = (arr.geom == XLMIMO_ULA) ? sqrt(fma(uq[0], uq[0], uq[2] * uq[2])) : fabs(uq[0]);
      scale = arr.beta0 * sqrt(xp * xq);
    }
    if (i > j) im = -im;  // G_ji = conj(G_ij)
    gram[(dp.gram_off + idx) * 2] = re * scale;
    gram[(dp.gram_off + idx) * 2 + 1] = im * scale;
  }
}

template <int NBMAX, typename T>
static int grid_for() {
  static int cached = 0;
  if (!cached) {
    int dev = 0, n_cu = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gram_exact<NBMAX, T>, kGramThreads, 0);
    cached = (n_cu > 0 ? n_cu : 256) * (per_cu > 0 ? per_cu : 1);
  }
  return cached;
}

int gram_exact_grid(int precision, int nb_max, int n_items) {
  int g;
  if (precision == XLMIMO_FP64) g = nb_max <= 2 ? grid_for<2, double>() : grid_for<4, double>();
  else g = nb_max <= 2 ? grid_for<2, float>() : grid_for<4, float>();
  return n_items < g ? n_items : g;
}

hipError_t launch_gram_exact(int precision, int nb_max, const ArrayK& arr, const DropK* d_drops, int n_drops,
                             const double* d_pos, const ItemK* d_items, int n_items, int* d_counter,
                             double* d_partials, double* d_gram, int grid, hipStream_t s) {
  if (n_drops == 0) return hipSuccess;
  k_reset_counter<<<1, 64, 0, s>>>(d_counter);
  if (grid < 1) grid = 1;
  if (precision == XLMIMO_FP64) {
    if (nb_max <= 2) k_gram_exact<2, double><<<grid, kGramThreads, 0, s>>>(arr, d_drops, d_pos, d_items, n_items, d_counter, d_partials);
    else k_gram_exact<4, double><<<grid, kGramThreads, 0, s>>>(arr, d_drops, d_pos, d_items, n_items, d_counter, d_partials);
    k_gram_finalize<double><<<n_drops, 256, 0, s>>>(arr, d_drops, d_pos, d_partials, d_gram);
  } else {
    if (nb_max <= 2) k_gram_exact<2, float><<<grid, kGramThreads, 0, s>>>(arr, d_drops, d_pos, d_items, n_items, d_counter, d_partials);
    else k_gram_exact<4, float><<<grid, kGramThreads, 0, s>>>(arr, d_drops, d_pos, d_items, n_items, d_counter, d_partials);
    k_gram_finalize<float><<<n_drops, 256, 0, s>>>(arr, d_drops, d_pos, d_partials, d_gram);
  }
  return hipGetLastError();
}

}  // namespace xl
