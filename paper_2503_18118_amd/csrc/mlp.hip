// Learned residual correction of the closed-form correlation (an MLP in BF16 on
// the matrix cores, FP32 accumulation), with training kernels.
//
// Not in the paper: the correction targets the regime where the paper notes the
// modified ZF is worse (before saturation, Sec. V-C).  Per user pair (i < j):
//   features  (r_i/50, theta_i/(pi/3), r_j/50, theta_j/(pi/3), log4 N - 6, d/lambda - 1/2)
//   basis     b_top, b_bot: end-element terms of the discrete sum, f e^{j phi} / D with
//             D = 1 - e^{-+ j phi' d} (geometric series of the locally linear phase),
//             regularised by the Fresnel scale eps^2 = d^2 |phi''| / (2 pi);
//             b_spm = e^{j phi(y*)} at the stationary point; phi(y) = (2 pi/lambda)(r_i(y) - r_j(y))
//   network   6 -> [Linear(w) + GELU] x depth -> Linear(7)
//   output    coefficients c_m (3 complex) and s = log sigma^2;
//             delta_rho = sum_m c_m b_m;  G_ij += delta_rho sqrt(G~_ii G~_jj)
//   loss      mean |target - delta_rho|^2 e^{-s} + s   (Gaussian negative log-likelihood)
//   optimiser Adam on FP32 master weights, BF16 copies for the matrix cores.
//
// GEMM: C[M x N] = sum_k A(m,k) B(k,n) on v_mfma_f32_16x16x32_bf16, 64 x 64 tiles
// per 256-thread workgroup (each wave 32 x 32 = 2 x 2 MFMA blocks), K in steps
// of 32 staged through LDS with k contiguous, operands with arbitrary strides
// (so the same kernel serves X W^T, dZ W and dZ^T X).  Epilogues fuse
// bias + GELU (forward), the last-layer bias, and GELU' (backward).
#include <hip/hip_bf16.h>

#include <algorithm>

#include "device_math.h"
#include "internal.h"
#include "pair_math.h"
#include "xlmimo.h"

namespace xl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TM = 64, TN = 64, TK = 32;
constexpr int LDS_K = TK + 8;  // row pitch in bf16 (80 bytes: 16-byte aligned operand reads)
constexpr double kPiD = 3.14159265358979323846264338327950288;

// GELU(z) = z Phi(z), Phi(z) = (1 + erf(z / sqrt 2)) / 2, with erfc(x) = t P(t) e^{-x^2},
// t = 1 / (1 + p x), x >= 0: the rational-exponential approximation 7.1.26 of
// Abramowitz and Stegun (Hastings), |error| <= 1.5e-7 in erf, far below the BF16
// rounding of the activations it feeds.  Written for Phi directly:
//   Q = erfc(|z| / sqrt 2) / 2 = t P(t) e^{-z^2/2} / 2,  Phi = 1 - Q (z >= 0), Q (z < 0)
// with p / sqrt 2 and the halved coefficients folded in: one reciprocal, one exp2.
// Then z Phi(z) = max(z, 0) - |z| Q for either sign of z.
struct GeluParts {
  float q;     // erfc(|z| / sqrt 2) / 2
  float e;     // e^{-z^2/2}
};
__device__ __forceinline__ GeluParts gelu_parts(float z) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.2316418882663604f, fabsf(z), 1.0f));
  const float p = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 0.5307027145f, -0.7265760135f), 0.7107068705f), -0.142248368f),
                           0.127414796f);
  GeluParts g;
  g.e = __builtin_amdgcn_exp2f(z * z * -0.7213475204444817f);
  g.q = p * g.e;
  return g;
}
// The forward value needs Q alone, taken without a reciprocal: Q(x) = 2^{P(x)}, P of
// degree 6 in x = min(|z|, 6) with P(0) = -1 (Q(0) = 1/2 exactly), fitted to log2 Q on
// [0, 6] for the error of x Q(x) (fit_gelu_tail.py); |error| in GELU <= 3.2e-7 in
// FP32, about the rounding of the result, 1.6e-7 relative for |z| < 0.01, and
// x Q(x) < 1e-8 |z| / 6 past the clamp.  Ten instructions, one of them an exp2,
// against thirteen with a reciprocal and an exp2 for the form above.
// Clamp and max(z, 0) as v_med3_f32: with IEEE min/max the compiler would first quiet
// the inputs (a v_max each) when z comes straight from the matrix core.
__device__ __forceinline__ float gelu(float z) {
  const float x = __builtin_amdgcn_fmed3f(fabsf(z), 0.0f, 6.0f);
  float p = fmaf(x, 2.992528485e-05f, -7.398832138e-04f);
  p = fmaf(p, x, 7.977489636e-03f);
  p = fmaf(p, x, -5.323822283e-02f);
  p = fmaf(p, x, -4.589156649e-01f);
  p = fmaf(p, x, -1.151147087e+00f);
  p = fmaf(p, x, -1.000000000e+00f);
  return fmaf(-fabsf(z), __builtin_amdgcn_exp2f(p), __builtin_amdgcn_fmed3f(z, 0.0f, 3.40282347e38f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  const GeluParts g = gelu_parts(z);
  const float phi = z >= 0.0f ? 1.0f - g.q : g.q;
  return fmaf(z * 0.3989422804014327f, g.e, phi);   // Phi(z) + z phi(z)
}

// Operand tiles: 64 rows (m of A, n of B) x TK = 32 k-values, staged in LDS with k
// contiguous (the MFMA operand layout).  Three ways to fetch a tile, chosen per operand
// on the host from its strides and alignment:
//   LOAD_K   k-contiguous rows, 16-byte aligned: thread t loads row t/4, k-values 8 (t%4) .. + 7
//            as one 16-byte vector (one 16-byte LDS store);
//   LOAD_R   row-contiguous (k strided), aligned: thread t loads rows 8 (t%8) .. + 7 at k = t/8
//            as one vector and stores them transposed (8 two-byte LDS stores);
//   LOAD_S   anything else: the LOAD_K pattern with element loads.
// Out-of-range elements load as zero (vector loads only where the whole vector is in range).
enum { LOAD_S = 0, LOAD_K = 1, LOAD_R = 2 };

template <int MODE>
__device__ __forceinline__ bf16x8 tile_fetch(const __bf16* __restrict__ P, int64_t p_r, int64_t p_k, int rows, int r0,
                                             int k0, int ke, int tid) {
  bf16x8 v;
  if constexpr (MODE == LOAD_R) {
    const int k = k0 + (tid >> 3), rc = r0 + 8 * (tid & 7);
    if (k < ke && rc + 8 <= rows) {
      v = *reinterpret_cast<const bf16x8*>(P + (int64_t)k * p_k + rc);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = (k < ke && rc + q < rows) ? P[(int64_t)k * p_k + rc + q] : (__bf16)0.0f;
    }
  } else {
    const int r = r0 + (tid >> 2), kc = k0 + 8 * (tid & 3);
    if (MODE == LOAD_K && r < rows && kc + 8 <= ke) {
      v = *reinterpret_cast<const bf16x8*>(P + (int64_t)r * p_r + kc);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[q] = (r < rows && kc + q < ke) ? P[(int64_t)r * p_r + (int64_t)(kc + q) * p_k] : (__bf16)0.0f;
    }
  }
  return v;
}

template <int MODE>
__device__ __forceinline__ void tile_store(__bf16* s, const bf16x8& v, int tid) {
  if constexpr (MODE == LOAD_R) {
    const int k = tid >> 3, rc = 8 * (tid & 7);
#pragma unroll
    for (int q = 0; q < 8; ++q) s[(rc + q) * LDS_K + k] = v[q];
  } else {
    *reinterpret_cast<bf16x8*>(&s[(tid >> 2) * LDS_K + 8 * (tid & 3)]) = v;
  }
}

// Epilogue of a (64 MT) x 64 tile.  The MFMAs take B's fragment as their first operand, so a
// 16x16 block comes out transposed: lane l, register r -> row l % 16, column 4 (l / 16) + r,
// i.e. each lane holds four consecutive columns of one row and writes them as one vector
// (16 bytes of FP32, 8 of BF16) wherever they are in range and aligned.
__device__ __forceinline__ bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }
__device__ __forceinline__ bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

template <int EPI, int MT>
__device__ __forceinline__ void gemm_store(const GemmArgs& g, const floatx4 (&acc)[2 * MT][2], int m0, int n0, int wm,
                                           int wn, int lane, int bz) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  const int64_t slice = g.row_sums ? (int64_t)g.M * g.ldo + g.M : (int64_t)g.M * g.ldo;
#pragma unroll
  for (int i = 0; i < 2 * MT; ++i) {
    const int row = m0 + wm + i * 16 + (lane & 15);
    if (row >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + j * 16 + 4 * (lane >> 4);
      const int64_t o = (int64_t)row * g.ldo + col;
      const floatx4 v = acc[i][j];
      const bool whole = col + 4 <= g.N;
      if constexpr (EPI == EPI_FWD_HIDDEN) {
        if (whole && aligned16(&g.bias[col]) && aligned8(&g.out_bf[o]) && (!g.Z || aligned16(&g.Z[o]))) {
          const floatx4 b = *reinterpret_cast<const floatx4*>(&g.bias[col]);
          const floatx4 z = v + b;
          if (g.Z) *reinterpret_cast<floatx4*>(&g.Z[o]) = z;
          const bf16x4 y = {(__bf16)gelu(z[0]), (__bf16)gelu(z[1]), (__bf16)gelu(z[2]), (__bf16)gelu(z[3])};
          *reinterpret_cast<bf16x4*>(&g.out_bf[o]) = y;
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (col + r >= g.N) continue;
            const float z = v[r] + g.bias[col + r];
            if (g.Z) g.Z[o + r] = z;
            g.out_bf[o + r] = (__bf16)gelu(z);
          }
        }
      } else if constexpr (EPI == EPI_FWD_OUT) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (col + r < g.N) g.out_f[o + r] = v[r] + g.bias[col + r];
      } else if constexpr (EPI == EPI_BWD_DX) {
        if (whole && aligned16(&g.Z[o]) && aligned8(&g.out_bf[o])) {
          const floatx4 z = *reinterpret_cast<const floatx4*>(&g.Z[o]);
          const bf16x4 d = {(__bf16)(v[0] * gelu_grad(z[0])), (__bf16)(v[1] * gelu_grad(z[1])),
                            (__bf16)(v[2] * gelu_grad(z[2])), (__bf16)(v[3] * gelu_grad(z[3]))};
          *reinterpret_cast<bf16x4*>(&g.out_bf[o]) = d;
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (col + r < g.N) g.out_bf[o + r] = (__bf16)(v[r] * gelu_grad(g.Z[o + r]));
        }
      } else {
        float* dst = g.out_f + (int64_t)bz * slice + o;
        if (whole && aligned16(dst)) {
          *reinterpret_cast<floatx4*>(dst) = v;
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (col + r < g.N) dst[r] = v[r];
        }
      }
    }
  }
}

// Double-buffered main loop: the next k-step's tiles are fetched into registers while the
// matrix cores work on the current one from LDS; one barrier per k-step.  A workgroup
// computes a (64 MT) x 64 tile; each of its 4 waves a (32 MT) x 32 block of 16x16 MFMA tiles.
template <int EPI, int AM, int BM, int MT>
__device__ __forceinline__ void gemm_block(const GemmArgs& g, int bx, int by, int bz) {
  constexpr int TMM = TM * MT;
  __shared__ __attribute__((aligned(16))) __bf16 sA[2][TMM * LDS_K];
  __shared__ __attribute__((aligned(16))) __bf16 sB[2][TN * LDS_K];
  constexpr bool RS = EPI == EPI_STORE_F32 && AM == LOAD_R;
  static_assert(!RS || MT == 1, "row sums with single row tiles");
  __shared__ float s_rs[RS ? 32 * TM : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = by * TMM, n0 = bx * TN;
  const int wm = (wave >> 1) * 32 * MT, wn = (wave & 1) * 32;
  floatx4 acc[2 * MT][2];
#pragma unroll
  for (int i = 0; i < 2 * MT; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  int kb = 0, ke = g.K;
  if (EPI == EPI_STORE_F32 && g.k_chunk > 0) {
    kb = bz * g.k_chunk;
    ke = min(g.K, kb + g.k_chunk);
  }
  // row sums of A over this slice (bias gradients), accumulated from the fetched tiles
  const bool row_sums = RS && g.row_sums && bx == 0;
  float rs[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

  bf16x8 va[MT], vb;
#pragma unroll
  for (int t = 0; t < MT; ++t) va[t] = tile_fetch<AM>(g.A, g.a_m, g.a_k, g.M, m0 + TM * t, kb, ke, tid);
  vb = tile_fetch<BM>(g.B, g.b_n, g.b_k, g.N, n0, kb, ke, tid);
#pragma unroll
  for (int t = 0; t < MT; ++t) tile_store<AM>(sA[0] + TM * t * LDS_K, va[t], tid);
  tile_store<BM>(sB[0], vb, tid);
  if constexpr (RS) {
    if (row_sums) {
#pragma unroll
      for (int q = 0; q < 8; ++q) rs[q] += (float)va[0][q];
    }
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kb; k0 < ke; k0 += TK) {
    const bool more = k0 + TK < ke;
    if (more) {
#pragma unroll
      for (int t = 0; t < MT; ++t) va[t] = tile_fetch<AM>(g.A, g.a_m, g.a_k, g.M, m0 + TM * t, k0 + TK, ke, tid);
      vb = tile_fetch<BM>(g.B, g.b_n, g.b_k, g.N, n0, k0 + TK, ke, tid);
    }
    const int kk = 8 * (lane >> 4);
    bf16x8 af[2 * MT], bfr[2];
#pragma unroll
    for (int i = 0; i < 2 * MT; ++i)
      af[i] = *reinterpret_cast<const bf16x8*>(&sA[buf][(wm + i * 16 + (lane & 15)) * LDS_K + kk]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      bfr[j] = *reinterpret_cast<const bf16x8*>(&sB[buf][(wn + j * 16 + (lane & 15)) * LDS_K + kk]);
#pragma unroll
    for (int i = 0; i < 2 * MT; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
    if (more) {
#pragma unroll
      for (int t = 0; t < MT; ++t) tile_store<AM>(sA[buf ^ 1] + TM * t * LDS_K, va[t], tid);
      tile_store<BM>(sB[buf ^ 1], vb, tid);
      if constexpr (RS) {
        if (row_sums) {
#pragma unroll
          for (int q = 0; q < 8; ++q) rs[q] += (float)va[0][q];
        }
      }
    }
    __syncthreads();
    buf ^= 1;
  }
  if constexpr (RS) {
    if (row_sums) {
      // thread t holds rows 8 (t%8) .. + 7 summed over k = t/8 (mod 32): fixed-order sum over t/8
#pragma unroll
      for (int q = 0; q < 8; ++q) s_rs[(tid >> 3) * TM + 8 * (tid & 7) + q] = rs[q];
      __syncthreads();
      if (tid < TM && m0 + tid < g.M) {
        float t = 0.f;
        for (int j = 0; j < 32; ++j) t += s_rs[j * TM + tid];
        g.out_f[(int64_t)bz * ((int64_t)g.M * g.ldo + g.M) + (int64_t)g.M * g.ldo + m0 + tid] = t;
      }
    }
  }
  gemm_store<EPI, MT>(g, acc, m0, n0, wm, wn, lane, bz);
}

template <int EPI, int AM, int BM, int MT>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  gemm_block<EPI, AM, BM, MT>(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Whole-K variant for K <= kKallMax (the layers' own GEMMs: forward and input gradients):
// every k-step's A and B tiles are fetched at once (one memory latency per tile instead of
// one per k-step, which dominates a 256-deep contraction), staged in LDS with k contiguous,
// then contracted.  K-contiguous operands only (LOAD_K), 16-byte aligned rows.
constexpr int kKallMax = 256;
constexpr int KALL_P = kKallMax + 8;   // LDS row pitch (bf16)
constexpr int64_t kKallMaxBlocks = 512;

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_kall(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 sA[TM * KALL_P];
  __shared__ __attribute__((aligned(16))) __bf16 sB[TN * KALL_P];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int K = g.K;
  constexpr int NKS = kKallMax / TK;
  bf16x8 va[NKS], vb[NKS];
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    if (ks * TK < K) {
      va[ks] = tile_fetch<LOAD_K>(g.A, g.a_m, g.a_k, g.M, m0, ks * TK, K, tid);
      vb[ks] = tile_fetch<LOAD_K>(g.B, g.b_n, g.b_k, g.N, n0, ks * TK, K, tid);
    }
  }
  const int r = tid >> 2, kc = 8 * (tid & 3);
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    if (ks * TK < K) {
      *reinterpret_cast<bf16x8*>(&sA[r * KALL_P + ks * TK + kc]) = va[ks];
      *reinterpret_cast<bf16x8*>(&sB[r * KALL_P + ks * TK + kc]) = vb[ks];
    }
  }
  __syncthreads();
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int kk = 8 * (lane >> 4);
  for (int k0 = 0; k0 < K; k0 += TK) {
    bf16x8 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) af[i] = *reinterpret_cast<const bf16x8*>(&sA[(wm + i * 16 + (lane & 15)) * KALL_P + k0 + kk]);
#pragma unroll
    for (int j = 0; j < 2; ++j) bfr[j] = *reinterpret_cast<const bf16x8*>(&sB[(wn + j * 16 + (lane & 15)) * KALL_P + k0 + kk]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
  }
  gemm_store<EPI, 1>(g, acc, m0, n0, wm, wn, lane, 0);
}

// Several split-K weight-gradient GEMMs in one launch: problem p owns the flat block range
// [first[p], first[p + 1]), laid out as its own (gx, gy, slices) grid.
template <int AM, int BM>
__global__ __launch_bounds__(256) void k_gemm_grouped(GemmGroup G) {
  const int b = blockIdx.x;
  int p = 0;
  while (p + 1 < G.n && b >= G.first[p + 1]) ++p;
  const int local = b - G.first[p];
  const int gx = G.gx[p], gy = G.gy[p];
  gemm_block<EPI_STORE_F32, AM, BM, 1>(G.g[p], local % gx, (local / gx) % gy, local / (gx * gy));
}

// out[i] = sum over splits of partial[split][i], in split order.
__global__ void k_reduce_splits(const float* __restrict__ partial, int splits, int64_t n, float* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.0f;
  for (int z = 0; z < splits; ++z) acc += partial[(int64_t)z * n + i];
  out[i] = acc;
}

// Fetch mode of an operand with row stride p_r and k stride p_k.
static int load_mode(const __bf16* P, int64_t p_r, int64_t p_k) {
  const bool aligned = ((uintptr_t)P & 15) == 0;
  if (p_k == 1 && p_r % 8 == 0 && aligned) return LOAD_K;
  if (p_r == 1 && p_k % 8 == 0 && aligned) return LOAD_R;
  return LOAD_S;
}

template <int EPI, int MT>
static void launch_modes_mt(const GemmArgs& g, dim3 grid, hipStream_t s) {
  const int am = load_mode(g.A, g.a_m, g.a_k), bm = load_mode(g.B, g.b_n, g.b_k);
#define XL_GEMM_CASE(A_, B_) \
  if (am == A_ && bm == B_) { k_gemm_bf16<EPI, A_, B_, MT><<<grid, 256, 0, s>>>(g); return; }
  XL_GEMM_CASE(LOAD_K, LOAD_K)
  XL_GEMM_CASE(LOAD_K, LOAD_R)
  XL_GEMM_CASE(LOAD_R, LOAD_R)
  XL_GEMM_CASE(LOAD_K, LOAD_S)
  XL_GEMM_CASE(LOAD_R, LOAD_S)
  XL_GEMM_CASE(LOAD_S, LOAD_K)
  XL_GEMM_CASE(LOAD_S, LOAD_R)
#undef XL_GEMM_CASE
  k_gemm_bf16<EPI, LOAD_S, LOAD_S, MT><<<grid, 256, 0, s>>>(g);
}

template <int EPI>
static void launch_modes(const GemmArgs& g, dim3 grid, hipStream_t s) {
  // (row tiles of 128, half the workgroups at batch 8192, measured 13 % slower per training step)
  launch_modes_mt<EPI, 1>(g, grid, s);
}

hipError_t launch_gemm_splitk_partials(const GemmArgs& g0, int splits, float* partial, int* slices, hipStream_t s) {
  GemmArgs g = g0;
  g.k_chunk = ((g.K + splits - 1) / splits + TK - 1) / TK * TK;
  splits = (g.K + g.k_chunk - 1) / g.k_chunk;
  g.out_f = partial;
  dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM, splits);
  if (g.row_sums && load_mode(g.A, g.a_m, g.a_k) != LOAD_R) return hipErrorInvalidValue;
  launch_modes<EPI_STORE_F32>(g, grid, s);
  *slices = splits;
  return hipGetLastError();
}

hipError_t launch_gemm_grouped_partials(const GemmArgs* gs, const int* splits, float* const* partials, int n,
                                       int* slices, hipStream_t s) {
  if (n < 1 || n > kMaxLayers) return hipErrorInvalidValue;
  GemmGroup G{};
  G.n = n;
  int total = 0;
  int am = -1, bm = -1;
  for (int p = 0; p < n; ++p) {
    GemmArgs g = gs[p];
    g.k_chunk = ((g.K + splits[p] - 1) / splits[p] + TK - 1) / TK * TK;
    slices[p] = (g.K + g.k_chunk - 1) / g.k_chunk;
    g.out_f = partials[p];
    const int a = load_mode(g.A, g.a_m, g.a_k), b = load_mode(g.B, g.b_n, g.b_k);
    if ((am >= 0 && a != am) || (bm >= 0 && b != bm)) return hipErrorInvalidValue;   // one fetch mode per launch
    am = a;
    bm = b;
    if (g.row_sums && a != LOAD_R) return hipErrorInvalidValue;
    G.g[p] = g;
    G.gx[p] = (g.N + TN - 1) / TN;
    G.gy[p] = (g.M + TM - 1) / TM;
    G.first[p] = total;
    total += G.gx[p] * G.gy[p] * slices[p];
  }
  G.first[n] = total;
  if (total == 0) return hipSuccess;
  if (am == LOAD_R && bm == LOAD_R) k_gemm_grouped<LOAD_R, LOAD_R><<<total, 256, 0, s>>>(G);
  else if (am == LOAD_R && bm == LOAD_K) k_gemm_grouped<LOAD_R, LOAD_K><<<total, 256, 0, s>>>(G);
  else if (am == LOAD_R) k_gemm_grouped<LOAD_R, LOAD_S><<<total, 256, 0, s>>>(G);
  else k_gemm_grouped<LOAD_S, LOAD_S><<<total, 256, 0, s>>>(G);
  return hipGetLastError();
}

hipError_t launch_gemm_splitk(const GemmArgs& g, int splits, float* partial, float* out, hipStream_t s) {
  int slices = 0;
  hipError_t e = launch_gemm_splitk_partials(g, splits, partial, &slices, s);
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)g.M * g.ldo + (g.row_sums ? g.M : 0);
  k_reduce_splits<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(partial, slices, n, out);
  return hipGetLastError();
}

// Gradient of parameter i from its layer's unreduced slices, summed in slice order
// (the order of k_reduce_splits).
__device__ __forceinline__ float layer_grad(const SplitLayers& L, const float* __restrict__ part, int64_t i) {
  int l = 0;
  while (l + 1 < L.n && i >= L.start[l + 1]) ++l;
  const int64_t nl = L.start[l + 1] - L.start[l];
  const float* p = part + L.part_off[l] + (i - L.start[l]);
  float acc = 0.0f;
  for (int z = 0; z < L.splits[l]; ++z) acc += p[(int64_t)z * nl];
  return acc;
}

__global__ void k_reduce_layers(SplitLayers L, const float* __restrict__ part, float* __restrict__ grad) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < L.start[L.n]) grad[i] = layer_grad(L, part, i);
}

hipError_t launch_reduce_layers(const SplitLayers& L, const float* part, float* grad, hipStream_t s) {
  const int64_t n = L.start[L.n];
  if (n > 0) k_reduce_layers<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(L, part, grad);
  return hipGetLastError();
}

hipError_t launch_gemm(int epi, const GemmArgs& g, hipStream_t s) {
  dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM);
  // whole-K staging while the grid fits the chip in one round (two 68 KB workgroups per CU);
  // larger grids hide the fetch latency better with more, smaller workgroups per CU
  if (epi != EPI_STORE_F32 && g.K <= kKallMax && (int64_t)grid.x * grid.y <= kKallMaxBlocks &&
      load_mode(g.A, g.a_m, g.a_k) == LOAD_K && load_mode(g.B, g.b_n, g.b_k) == LOAD_K) {
    switch (epi) {
      case EPI_FWD_HIDDEN: k_gemm_kall<EPI_FWD_HIDDEN><<<grid, 256, 0, s>>>(g); break;
      case EPI_FWD_OUT: k_gemm_kall<EPI_FWD_OUT><<<grid, 256, 0, s>>>(g); break;
      default: k_gemm_kall<EPI_BWD_DX><<<grid, 256, 0, s>>>(g); break;
    }
    return hipGetLastError();
  }
  switch (epi) {
    case EPI_FWD_HIDDEN: launch_modes<EPI_FWD_HIDDEN>(g, grid, s); break;
    case EPI_FWD_OUT: launch_modes<EPI_FWD_OUT>(g, grid, s); break;
    case EPI_BWD_DX: launch_modes<EPI_BWD_DX>(g, grid, s); break;
    default: launch_modes<EPI_STORE_F32>(g, grid, s); break;
  }
  return hipGetLastError();
}

// e^{j 2 pi u} for a phase u in turns (FP64 reduction, FP64 Taylor sin/cos).
__device__ __forceinline__ void phasor_turns(double u, float& re, float& im) {
  const double v = 2.0 * u;  // half turns
  const double q = __builtin_rint(v);
  double ns, c;
  sincos_half(v - q, ns, c);
  const double sg = (((long long)q) & 1) ? -1.0 : 1.0;
  re = (float)(sg * c);
  im = (float)(-sg * ns);
}

// The residual is predicted on top of the analytic end correction: the
// coefficients of the basis phasors (top end, bottom end, stationary point) are
// basis_c0 + the network's outputs, so an all-zero output is the discrete sum's
// two end terms added to the closed form, and the network only learns how far
// the best coefficients lie from them.
__device__ __forceinline__ float basis_c0(int m) { return m < 2 ? 1.0f : 0.0f; }

__global__ __launch_bounds__(256) void k_pair_inputs(ArrayK arr, const DropK* __restrict__ drops,
                                                      const double* __restrict__ pos,
                                                      const double* __restrict__ gram_cf,
                                                      const double* __restrict__ gram_exact,
                                                      __bf16* __restrict__ feat, float* __restrict__ aux,
                                                      float* __restrict__ target, int32_t* __restrict__ pmap) {
  const DropK dp = drops[blockIdx.x];
  const int K = dp.k;
  const int np = K * (K - 1) / 2;
  const double lam = arr.lambda;
  const double ytop = 0.5 * (double)(dp.n_elems - 1) * arr.spacing;
  // per user, once per drop: perpendicular distance and position, the two user features, and
  // at each array end (top, bottom) the distance r_e, (y_e - y) / r_e and x^2 / r_e^3
  constexpr int kU = 10;
  __shared__ double s_user[XLMIMO_MAX_USERS * kU];
  for (int u = threadIdx.x; u < K; u += blockDim.x) {
    const double* pu = pos + (dp.user_off + u) * 3;
    const double x = sqrt(fma(pu[0], pu[0], pu[2] * pu[2])), y = pu[1];
    double* su = s_user + u * kU;
    su[0] = x;
    su[1] = y;
    su[2] = sqrt(x * x + y * y) / 50.0;
    su[3] = atan2(y, x) / (kPiD / 3.0);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const double d = (e == 0 ? ytop : -ytop) - y;
      const double r = sqrt(fma(d, d, x * x));
      su[4 + 3 * e] = r;
      su[5 + 3 * e] = d / r;
      su[6 + 3 * e] = x * x / (r * r * r);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < np; t += blockDim.x) {
    int i = 0, rem = t;
    while (rem >= K - 1 - i) {
      rem -= K - 1 - i;
      ++i;
    }
    const int j = i + 1 + rem;
    const int64_t p = dp.pair_off + t;
    const double* si = s_user + i * kU;
    const double* sj = s_user + j * kU;
    const double xi = si[0], yi = si[1];
    const double xj = sj[0], yj = sj[1];
    const double f[8] = {si[2], si[3], sj[2], sj[3],
                         log((double)dp.n_elems) / log(4.0) - 6.0, arr.spacing / lam - 0.5, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 8; ++q) feat[p * 8 + q] = (__bf16)(float)f[q];
    auto dphase = [&](double y) {  // (r_i(y) - r_j(y)) / lambda in turns
      const double di = y - yi, dj = y - yj;
      return (sqrt(fma(di, di, xi * xi)) - sqrt(fma(dj, dj, xj * xj))) * arr.inv_lambda;
    };
    const double* gc = gram_cf + 2 * dp.gram_off;
    const double scale = sqrt(gc[2 * (i * K + i)] * gc[2 * (j * K + j)]);
    const double kw = 2.0 * kPiD * arr.inv_lambda;
    const double c_fs = (lam / (4.0 * kPiD)) * (lam / (4.0 * kPiD));
    // End-element term of the discrete sum: f e^{j phi} conj(D) / (|D|^2 + eps^2),
    // D = 1 - e^{-j sign phi' d}, eps^2 = d^2 |phi''| / (2 pi), in correlation units
    // (end e: 0 top, 1 bottom, from the per-user values above).
    auto end_term = [&](int e, double sign, float& br, float& bi) {
      const double ra = si[4 + 3 * e], rb = sj[4 + 3 * e];
      const double d1 = kw * (si[5 + 3 * e] - sj[5 + 3 * e]);
      const double d2 = kw * (si[6 + 3 * e] - sj[6 + 3 * e]);
      const double ang = sign * d1 * arr.spacing;
      const double dre = 1.0 - cos(ang), dim = sin(ang);
      const double den = dre * dre + dim * dim + arr.spacing * arr.spacing * fabs(d2) / (2.0 * kPiD);
      const double amp = (arr.amp == XLMIMO_AMP_FREESPACE) ? c_fs / (ra * rb)
                                                           : arr.beta0 * sqrt(xi * xj) / ((ra * rb) * sqrt(ra * rb));
      float pr, pi;
      phasor_turns((ra - rb) * arr.inv_lambda, pr, pi);
      const double g = amp / (den * scale);
      // (pr + j pi)(dre - j dim)
      br = (float)(g * ((double)pr * dre + (double)pi * dim));
      bi = (float)(g * ((double)pi * dre - (double)pr * dim));
    };
    float pr, pi;
    end_term(0, 1.0, pr, pi);
    aux[p * 8 + 0] = pr;
    aux[p * 8 + 1] = pi;
    end_term(1, -1.0, pr, pi);
    aux[p * 8 + 2] = pr;
    aux[p * 8 + 3] = pi;
    if (xi != xj) {
      phasor_turns(dphase((yi * xj - xi * yj) / (xj - xi)), pr, pi);
    } else {
      pr = 1.0f;
      pi = 0.0f;
    }
    aux[p * 8 + 4] = pr;
    aux[p * 8 + 5] = pi;
    {
      // pairs the base closed form evaluates numerically (variants GATED_QUAD, UNIFORM: slow-phase
      // pairs and broad stationary zones) are not corrected by the network
      const PairGeom pg{xi, yi, xj, yj, kw, arr.inv_lambda, arr.amp, arr.beta0, c_fs};
      int panels = 0;
      if (numeric_route(pg, dp.n_elems, arr.spacing, 64, panels) != ROUTE_NONE) {
#pragma unroll
        for (int q = 0; q < 6; ++q) aux[p * 8 + q] = 0.0f;
      }
    }
    aux[p * 8 + 6] = (float)scale;
    aux[p * 8 + 7] = 0.0f;
    if (target != nullptr) {
      const double* ge = gram_exact + 2 * dp.gram_off;
      const double eii = ge[2 * (i * K + i)], ejj = ge[2 * (j * K + j)];
      const double se = sqrt(eii * ejj);
      target[p * 2 + 0] = (float)(ge[2 * (i * K + j)] / se - gc[2 * (i * K + j)] / scale);
      target[p * 2 + 1] = (float)(ge[2 * (i * K + j) + 1] / se - gc[2 * (i * K + j) + 1] / scale);
    }
    pmap[p * 2 + 0] = (int32_t)blockIdx.x;
    pmap[p * 2 + 1] = i * XLMIMO_MAX_USERS + j;
  }
}

hipError_t launch_pair_inputs(const ArrayK& arr, const DropK* d_drops, int n_drops, const double* d_pos,
                              const double* d_cf, const double* d_exact, __bf16* feat, float* aux, float* target,
                              int32_t* pmap, hipStream_t s) {
  if (n_drops == 0) return hipSuccess;
  k_pair_inputs<<<n_drops, 256, 0, s>>>(arr, d_drops, d_pos, d_cf, d_exact, feat, aux, target, pmap);
  return hipGetLastError();
}

// Loss head: per-sample NLL and its gradient with respect to the 7 outputs
// (scaled by 1/n); per-block partial loss sums in fixed order.
__global__ __launch_bounds__(256) void k_mlp_head(int64_t n, const float* __restrict__ out,
                                                  const float* __restrict__ aux, const float* __restrict__ target,
                                                  __bf16* __restrict__ dout, double* __restrict__ partial) {
  __shared__ double s_sum[256];
  double acc = 0.0;
  const float inv_n = 1.0f / (float)n;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const float* o = out + p * 7;
    const float* a = aux + p * 8;
    float prr = 0.f, pii = 0.f;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const float cr = o[2 * m] + basis_c0(m);
      prr += cr * a[2 * m] - o[2 * m + 1] * a[2 * m + 1];
      pii += cr * a[2 * m + 1] + o[2 * m + 1] * a[2 * m];
    }
    const float s = o[6];
    const float er = target[2 * p] - prr, ei = target[2 * p + 1] - pii;
    const float w = expf(-s);
    const float e2 = er * er + ei * ei;
    acc += (double)(e2 * w + s);
    const float gpr = -2.0f * er * w * inv_n, gpi = -2.0f * ei * w * inv_n;
    __bf16* d = dout + p * kDoutPitch;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      d[2 * m] = (__bf16)(gpr * a[2 * m] + gpi * a[2 * m + 1]);
      d[2 * m + 1] = (__bf16)(-gpr * a[2 * m + 1] + gpi * a[2 * m]);
    }
    d[6] = (__bf16)((1.0f - e2 * w) * inv_n);
    d[7] = (__bf16)0.0f;
  }
  s_sum[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s_sum[0];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int n_part, int64_t n,
                                                      double* __restrict__ loss) {
  __shared__ double s_sum[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n_part; i += 256) acc += partial[i];
  s_sum[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = s_sum[0] / (double)n;
}

hipError_t launch_mlp_head(int64_t n, const float* out, const float* aux, const float* target, __bf16* dout,
                           double* partial, double* loss, hipStream_t s) {
  k_mlp_head<<<kMlpHeadBlocks, 256, 0, s>>>(n, out, aux, target, dout, partial);
  if (loss != nullptr) k_sum_partials<<<1, 256, 0, s>>>(partial, kMlpHeadBlocks, n, loss);
  return hipGetLastError();
}

// Layer of parameter i and, for a weight, its index in the layer's transposed [in][out] copy
// (-1 for a bias).
__device__ __forceinline__ int layer_of(const SplitLayers& L, int64_t i) {
  int l = 0;
  while (l + 1 < L.n && i >= L.start[l + 1]) ++l;
  return l;
}
__device__ __forceinline__ int64_t transposed_index(const SplitLayers& L, int l, int64_t i) {
  const int64_t j = i - L.start[l];
  const int in = L.in_dim[l];
  const int64_t o = (L.start[l + 1] - L.start[l]) / (in + 1);
  if (j >= o * in) return -1;
  const int64_t oi = j / in, ii = j - oi * in;
  return L.start[l] + ii * o + oi;
}

// Adam with the gradient summed from the layers' split-K slices (the reduction and the
// update in one pass over the parameters), or taken from grad; block 0 also finishes the
// loss (k_sum_partials).
__global__ __launch_bounds__(256) void k_adam_layers(SplitLayers L, const float* __restrict__ part,
                                                     const float* __restrict__ grad, int64_t n, float* __restrict__ w,
                                                     float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                     float b2, float eps, float bc1, float bc2,
                                                     __bf16* __restrict__ wbf, __bf16* __restrict__ wbf_t,
                                                     const double* __restrict__ loss_part, int n_loss_part,
                                                     int64_t n_pairs, double* __restrict__ loss) {
  if (blockIdx.x == 0 && loss != nullptr) {
    __shared__ double s_sum[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n_loss_part; i += 256) acc += loss_part[i];
    s_sum[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss = s_sum[0] / (double)n_pairs;
  }
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = part != nullptr ? layer_grad(L, part, i) : grad[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  w[i] = wi;
  wbf[i] = (__bf16)wi;
  const int64_t t = transposed_index(L, layer_of(L, i), i);
  if (t >= 0) wbf_t[t] = (__bf16)wi;
}

hipError_t launch_adam_layers(const SplitLayers& L, const float* part, const float* grad, int64_t n, float* w,
                              float* m, float* v, float lr, float b1, float b2, float eps, float bc1, float bc2,
                              __bf16* wbf, __bf16* wbf_t, const double* loss_part, int n_loss_part, int64_t n_pairs,
                              double* loss, hipStream_t s) {
  if (n > 0 || loss != nullptr)
    k_adam_layers<<<(unsigned)std::max<int64_t>(1, (n + 255) / 256), 256, 0, s>>>(
        L, part, grad, n, w, m, v, lr, b1, b2, eps, bc1, bc2, wbf, wbf_t, loss_part, n_loss_part, n_pairs, loss);
  return hipGetLastError();
}

__global__ void k_weights_t(SplitLayers L, const float* __restrict__ w, __bf16* __restrict__ wbf_t) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= L.start[L.n]) return;
  const int64_t t = transposed_index(L, layer_of(L, i), i);
  if (t >= 0) wbf_t[t] = (__bf16)w[i];
}

hipError_t launch_weights_t(const SplitLayers& L, const float* w, __bf16* wbf_t, hipStream_t s) {
  const int64_t n = L.start[L.n];
  if (n > 0) k_weights_t<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(L, w, wbf_t);
  return hipGetLastError();
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ w, __bf16* __restrict__ wbf) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) wbf[i] = (__bf16)w[i];
}

hipError_t launch_to_bf16(int64_t n, const float* w, __bf16* wbf, hipStream_t s) {
  k_to_bf16<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, w, wbf);
  return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n > 0) k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

__global__ void k_or_flags(int32_t* status, const int32_t* flags, int64_t n, int32_t bit) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && flags[i]) status[i] |= bit;
}

hipError_t launch_or_flags(int32_t* status, const int32_t* flags, int64_t n, int32_t bit, hipStream_t s) {
  if (n > 0) k_or_flags<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(status, flags, n, bit);
  return hipGetLastError();
}

// Apply the predicted residual to the closed-form Gram and flag drops whose
// predicted log-variance exceeds the threshold (they are recomputed exactly).
__global__ void k_mlp_apply(int64_t n, const float* __restrict__ out, const float* __restrict__ aux,
                            const int32_t* __restrict__ pmap, const DropK* __restrict__ drops,
                            double* __restrict__ gram, int32_t* __restrict__ flags, GateK gate) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float* o = out + p * 7;
  const float* a = aux + p * 8;
  double pr = 0.0, pi = 0.0;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double cr = (double)o[2 * m] + (double)basis_c0(m);
    pr += cr * a[2 * m] - (double)o[2 * m + 1] * a[2 * m + 1];
    pi += cr * a[2 * m + 1] + (double)o[2 * m + 1] * a[2 * m];
  }
  const int d = pmap[2 * p];
  const int i = pmap[2 * p + 1] / XLMIMO_MAX_USERS, j = pmap[2 * p + 1] % XLMIMO_MAX_USERS;
  const DropK dp = drops[d];
  const double sc = (double)a[6];
  double* gij = gram + 2 * (dp.gram_off + (int64_t)i * dp.k + j);
  double* gji = gram + 2 * (dp.gram_off + (int64_t)j * dp.k + i);
  gij[0] += pr * sc;
  gij[1] += pi * sc;
  gji[0] += pr * sc;
  gji[1] -= pi * sc;
  float thr = gate.cap;
  for (int b = 0; b < gate.n_bins; ++b) {
    if ((int64_t)dp.n_elems <= gate.n_upper[b]) {
      thr = fminf(thr, gate.thr[b]);
      break;
    }
  }
  if (!(o[6] <= thr)) atomicOr(&flags[d], 1);
}

hipError_t launch_mlp_apply(int64_t n, const float* out, const float* aux, const int32_t* pmap, const DropK* d_drops,
                            double* gram, int32_t* flags, const GateK& gate, hipStream_t s) {
  if (n > 0) k_mlp_apply<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, out, aux, pmap, d_drops, gram, flags, gate);
  return hipGetLastError();
}

// Fused forward pass for inference: one workgroup of NW waves carries a tile of
// 16 NB pairs through every layer.  Activations stay in LDS (bf16, one buffer of
// 16 NB x (W + 8)); weights are read from L2 as 16-byte fragments straight into
// MFMA operand registers (W[o][k] is k-contiguous), and each fragment feeds NB
// MFMAs: the weight traffic per pair falls as the tile grows (W = 256 and W = 128 run
// 128-pair tiles: 0.86 against 0.99 ms per 10^6 pairs with 64-pair tiles at W = 256, depth 4;
// 0.30 against 0.32 ms at W = 128, depth 4; W = 64 keeps 64-pair tiles, 0.11 ms against 0.12
// and 0.14 with 128 and 256 pairs).  Wave w
// owns output columns [w W/NW, (w+1) W/NW) of the hidden layers and row blocks
// w, w + NW, ... of the output layer.
// TRAIN: also store each hidden layer's pre-activation (FP32) and GELU output (BF16) for the
// backward pass (keep); the stores leave from the registers the epilogue already holds (four
// consecutive features of one pair per lane: one 16-byte and one 8-byte store).
template <int W, int NB, int NW, bool TRAIN = false>
__global__ __launch_bounds__(64 * NW) void k_mlp_fused_forward(int64_t n, int depth, const __bf16* __restrict__ feat,
                                                           const __bf16* __restrict__ wbf,
                                                           const float* __restrict__ master,
                                                           const int64_t* __restrict__ offs, float* __restrict__ out,
                                                           FwdKeep keep) {
  // Activations resident in one LDS buffer (pair-major, features contiguous).  Hidden layers run as
  // out^T = W act^T: the weights are the MFMA's A operand (16 features x 32 k), the activations its B
  // operand (32 k x 16 pairs), so each lane's four results are four consecutive features of one pair
  // and leave in one 8-byte LDS store.
  constexpr int P = W + 8;           // LDS row pitch (bf16): 16-byte aligned rows
  constexpr int FB = W / (16 * NW);  // 16-feature blocks per wave
  __shared__ __attribute__((aligned(16))) __bf16 act[16 * NB * P];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * (16 * NB);
  const int kg = lane >> 4, li = lane & 15;
  const bf16x8 zero8 = {};

  // layer-0 input: 8 feature slots (6 used) per pair, zero up to K = 32
  for (int i = tid; i < 16 * NB * 32; i += 64 * NW) {
    const int r = i >> 5, k = i & 31;
    act[r * P + k] = (k < 8 && row0 + r < n) ? feat[(row0 + r) * 8 + k] : (__bf16)0.0f;
  }
  __syncthreads();

  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  // The weights of layer l's first two k-steps are in flight before its k-loop starts (for l > 0 they
  // are loaded while layer l - 1 finishes); inside the loop they run two k-steps ahead.
  auto load_w = [&](int l, int kk, bf16x8 (&wf)[FB]) {
    const __bf16* Wl = wbf + offs[2 * l];
#pragma unroll
    for (int i = 0; i < FB; ++i) {
      const int f = wave * (W / NW) + i * 16 + li;
      if (l == 0) {
        bf16x8 v = zero8;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (kk + q < XLMIMO_MLP_IN) v[q] = Wl[f * XLMIMO_MLP_IN + kk + q];
        wf[i] = v;
      } else {
        wf[i] = *reinterpret_cast<const bf16x8*>(&Wl[(int64_t)f * W + kk]);
      }
    }
  };
  bf16x8 wcur[FB], wn1[FB], wn2[FB];
#pragma unroll
  for (int i = 0; i < FB; ++i) wn1[i] = wn2[i] = zero8;   // layer 0 has a single k-step
  load_w(0, 8 * kg, wcur);
  for (int l = 0; l < depth; ++l) {  // hidden layers
    const int K = (l == 0) ? 32 : W;
    const float* bl = master + offs[2 * l + 1];
    // the sums start at the bias: the first k-step's products accumulate onto it (the bias is
    // that MFMA's addend), with no copies and no add in the epilogue
    floatx4 acc[FB][NB];
    {
      const int kk = 8 * kg;
      if (64 < K) load_w(l, kk + 64, wn2);
      bf16x8 af[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) af[j] = *reinterpret_cast<const bf16x8*>(&act[(j * 16 + li) * P + kk]);
#pragma unroll
      for (int i = 0; i < FB; ++i) {
        const int f0 = wave * (W / NW) + i * 16 + 4 * kg;
        const floatx4 bv = {bl[f0], bl[f0 + 1], bl[f0 + 2], bl[f0 + 3]};
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wcur[i], af[j], bv, 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < FB; ++i) {
        wcur[i] = wn1[i];
        wn1[i] = wn2[i];
      }
    }
    // the remaining k-steps (K = W past layer 0), unrolled so that the three weight
    // stages rotate by renaming rather than by register copies
    if (K > 32) {
#pragma unroll
      for (int k0 = 32; k0 < W; k0 += 32) {
        const int kk = k0 + 8 * kg;
        if (k0 + 64 < W) load_w(l, kk + 64, wn2);
        bf16x8 af[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) af[j] = *reinterpret_cast<const bf16x8*>(&act[(j * 16 + li) * P + kk]);
#pragma unroll
        for (int i = 0; i < FB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wcur[i], af[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < FB; ++i) {
          wcur[i] = wn1[i];
          wn1[i] = wn2[i];
        }
      }
    }
    if (l + 1 < depth) {   // the next layer's first two k-steps, in flight during this epilogue
      load_w(l + 1, 8 * kg, wcur);
      load_w(l + 1, 32 + 8 * kg, wn1);
    }
    // GELU into packed BF16 before the barrier; only the stores wait for the other waves
    bf16x4 outv[FB][NB];
#pragma unroll
    for (int i = 0; i < FB; ++i) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        outv[i][j][0] = (__bf16)gelu(acc[i][j][0]);
        outv[i][j][1] = (__bf16)gelu(acc[i][j][1]);
        outv[i][j][2] = (__bf16)gelu(acc[i][j][2]);
        outv[i][j][3] = (__bf16)gelu(acc[i][j][3]);
      }
    }
    if constexpr (TRAIN) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int64_t row = row0 + j * 16 + li;
        if (row < n) {
#pragma unroll
          for (int i = 0; i < FB; ++i) {
            const int f0 = wave * (W / NW) + i * 16 + 4 * kg;
            *reinterpret_cast<floatx4*>(&keep.z[l][row * W + f0]) = acc[i][j];
            *reinterpret_cast<bf16x4*>(&keep.x[l + 1][row * W + f0]) = outv[i][j];
          }
        }
      }
    }
    __syncthreads();   // every wave has read this layer's input
#pragma unroll
    for (int i = 0; i < FB; ++i) {
      const int f0 = wave * (W / NW) + i * 16 + 4 * kg;
#pragma unroll
      for (int j = 0; j < NB; ++j) *reinterpret_cast<bf16x4*>(&act[(j * 16 + li) * P + f0]) = outv[i][j];
    }
    __syncthreads();
  }

  // output layer: XLMIMO_MLP_OUT columns (one 16-column block), wave w takes row blocks w, w + NW, ...
  {
    const __bf16* Wl = wbf + offs[2 * depth];
    const float* bl = master + offs[2 * depth + 1];
    for (int rb = wave; rb < NB; rb += NW) {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < W; k0 += 32) {
        const int kk = k0 + 8 * kg;
        const bf16x8 af = *reinterpret_cast<const bf16x8*>(&act[(rb * 16 + li) * P + kk]);
        const bf16x8 bfr = (li < XLMIMO_MLP_OUT) ? *reinterpret_cast<const bf16x8*>(&Wl[(int64_t)li * W + kk]) : zero8;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, acc, 0, 0, 0);
      }
      if (li < XLMIMO_MLP_OUT) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = row0 + rb * 16 + 4 * kg + r;
          if (row < n) out[row * XLMIMO_MLP_OUT + li] = acc[r] + bl[li];
        }
      }
    }
  }
}

// The training step's input-gradient chain, fused like the forward: one workgroup of NW waves
// carries a tile of 16 NB pairs from the output gradient down to layer 1, the current gradient at
// the pre-activation (BF16, as the layer GEMMs round it) in one LDS buffer.  Layer l's product
// dA = dZ[l] W[l] runs as dA^T = W[l]^T dZ[l]^T: the transposed weights (k = output index
// contiguous) are the MFMA's A operand, the LDS gradient its B operand, so each lane's four results
// are four consecutive input features of one pair, multiplied by GELU'(z) of the same four features
// (one 16-byte load of the stored pre-activation) and stored as four BF16.  Wave w owns input
// features [w W/NW, (w+1) W/NW); the output layer's 7 rows enter as K = 32 with zeros beyond.
template <int W, int NB, int NW>
__global__ __launch_bounds__(64 * NW) void k_mlp_fused_train_backward(int64_t n, int depth,
                                                                  const __bf16* __restrict__ dout,
                                                                  const __bf16* __restrict__ wbf_t,
                                                                  const int64_t* __restrict__ offs, BwdKeep keep) {
  constexpr int P = W + 8;
  constexpr int FB = W / (16 * NW);
  __shared__ __attribute__((aligned(16))) __bf16 grad[16 * NB * P];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * (16 * NB);
  const int kg = lane >> 4, li = lane & 15;
  const bf16x8 zero8 = {};
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

  // the output gradient: 7 values per pair (pitch kDoutPitch), zero up to K = 32
  for (int i = tid; i < 16 * NB * 32; i += 64 * NW) {
    const int r = i >> 5, k = i & 31;
    grad[r * P + k] = (k < XLMIMO_MLP_OUT && row0 + r < n) ? dout[(row0 + r) * kDoutPitch + k] : (__bf16)0.0f;
  }
  __syncthreads();

  // W[l]^T fragment: input feature f, output indices kk .. kk + 7
  auto load_wt = [&](int l, int kk, bf16x8 (&wf)[FB]) {
    const __bf16* Wt = wbf_t + offs[2 * l];
#pragma unroll
    for (int i = 0; i < FB; ++i) {
      const int f = wave * (W / NW) + i * 16 + li;
      if (l == depth) {   // the output layer: W^T is W x 7
        bf16x8 v = zero8;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (kk + q < XLMIMO_MLP_OUT) v[q] = Wt[f * XLMIMO_MLP_OUT + kk + q];
        wf[i] = v;
      } else {
        wf[i] = *reinterpret_cast<const bf16x8*>(&Wt[(int64_t)f * W + kk]);
      }
    }
  };
  bf16x8 wcur[FB], wnext[FB];
  load_wt(depth, 8 * kg, wcur);
  for (int l = depth; l >= 1; --l) {
    const int K = (l == depth) ? 32 : W;
    floatx4 acc[FB][NB];
#pragma unroll
    for (int i = 0; i < FB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
      const int kk = k0 + 8 * kg;
      if (k0 + 32 < K) load_wt(l, kk + 32, wnext);
      bf16x8 af[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) af[j] = *reinterpret_cast<const bf16x8*>(&grad[(j * 16 + li) * P + kk]);
#pragma unroll
      for (int i = 0; i < FB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wcur[i], af[j], acc[i][j], 0, 0, 0);
      if (k0 + 32 < K) {
#pragma unroll
        for (int i = 0; i < FB; ++i) wcur[i] = wnext[i];
      }
    }
    if (l > 1) load_wt(l - 1, 8 * kg, wcur);   // in flight during the epilogue
    // dZ[l - 1] = dA * GELU'(z[l - 1]), rounded to BF16
    const float* zl = keep.z[l - 1];
    bf16x4 outv[FB][NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int64_t row = row0 + j * 16 + li;
#pragma unroll
      for (int i = 0; i < FB; ++i) {
        const int f0 = wave * (W / NW) + i * 16 + 4 * kg;
        const floatx4 zv = row < n ? *reinterpret_cast<const floatx4*>(&zl[row * W + f0]) : floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) outv[i][j][c] = (__bf16)(acc[i][j][c] * gelu_grad(zv[c]));
      }
    }
    __syncthreads();   // every wave has read this layer's gradient
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int64_t row = row0 + j * 16 + li;
#pragma unroll
      for (int i = 0; i < FB; ++i) {
        const int f0 = wave * (W / NW) + i * 16 + 4 * kg;
        *reinterpret_cast<bf16x4*>(&grad[(j * 16 + li) * P + f0]) = outv[i][j];
        if (row < n) *reinterpret_cast<bf16x4*>(&keep.dz[l - 1][row * W + f0]) = outv[i][j];
      }
    }
    __syncthreads();
  }
}

hipError_t launch_mlp_fused_forward(int width, int depth, int64_t n, const __bf16* feat, const __bf16* wbf,
                                    const float* master, const int64_t* d_offs, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 63) / 64);
  const unsigned grid2 = (unsigned)((n + 127) / 128);
  const FwdKeep none{};
  if (width == 256) k_mlp_fused_forward<256, 8, 4><<<grid2, 256, 0, s>>>(n, depth, feat, wbf, master, d_offs, out, none);
  else if (width == 128) k_mlp_fused_forward<128, 8, 4><<<grid2, 256, 0, s>>>(n, depth, feat, wbf, master, d_offs, out, none);
  else if (width == 64) k_mlp_fused_forward<64, 4, 4><<<grid, 256, 0, s>>>(n, depth, feat, wbf, master, d_offs, out, none);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// Training batches are 10^3-10^5 pairs, so the tiles are small: at width 256, 8 waves of 32
// features over 64 pairs from 16384 pairs on (256 workgroups and more), 32 pairs below (batch
// 16384: 125 TFLOP/s for the whole step against 115 with 4 waves of 64 features; batch 8192:
// 91 against 80 with 64-pair tiles); at width 128, 8 waves of 16 features over 32 pairs (batch
// 16384, depth 4: 64 TFLOP/s against 58 with 4 waves over 64 pairs); at width 64, 4 waves of 16
// features over 32 pairs (16500 against 15400 steps/s over 64 pairs).
hipError_t launch_mlp_fused_train_forward(int width, int depth, int64_t n, const __bf16* feat, const __bf16* wbf,
                                          const float* master, const int64_t* d_offs, const FwdKeep& keep,
                                          float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (depth < 1 || depth >= kMaxLayers) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((n + 63) / 64), grid32 = (unsigned)((n + 31) / 32);
  if (width == 256 && n >= 16384)
    k_mlp_fused_forward<256, 4, 8, true><<<grid, 512, 0, s>>>(n, depth, feat, wbf, master, d_offs, out, keep);
  else if (width == 256) k_mlp_fused_forward<256, 2, 8, true><<<grid32, 512, 0, s>>>(n, depth, feat, wbf, master, d_offs, out, keep);
  else if (width == 128) k_mlp_fused_forward<128, 2, 8, true><<<grid32, 512, 0, s>>>(n, depth, feat, wbf, master, d_offs, out, keep);
  else if (width == 64) k_mlp_fused_forward<64, 2, 4, true><<<grid32, 256, 0, s>>>(n, depth, feat, wbf, master, d_offs, out, keep);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_mlp_fused_train_backward(int width, int depth, int64_t n, const __bf16* dout, const __bf16* wbf_t,
                                           const int64_t* d_offs, const BwdKeep& keep, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (depth < 1 || depth >= kMaxLayers) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((n + 63) / 64), grid32 = (unsigned)((n + 31) / 32);
  if (width == 256 && n >= 16384)   // the tiles of the forward above
    k_mlp_fused_train_backward<256, 4, 8><<<grid, 512, 0, s>>>(n, depth, dout, wbf_t, d_offs, keep);
  else if (width == 256) k_mlp_fused_train_backward<256, 2, 8><<<grid32, 512, 0, s>>>(n, depth, dout, wbf_t, d_offs, keep);
  else if (width == 128) k_mlp_fused_train_backward<128, 2, 8><<<grid32, 512, 0, s>>>(n, depth, dout, wbf_t, d_offs, keep);
  else if (width == 64) k_mlp_fused_train_backward<64, 2, 4><<<grid32, 256, 0, s>>>(n, depth, dout, wbf_t, d_offs, keep);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace xl
