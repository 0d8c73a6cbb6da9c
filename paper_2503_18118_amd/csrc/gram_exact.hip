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
// Channel entry (one lane, one user, one element), coordinates scaled so that
// the distance r is the phase in turns (FP32C) or half turns (FP64):
//   r^2 = (y_u - y_e)^2 (+ (z_u - z_e)^2) + x_u^2                 FP64
//   y0 = rsq(r^2) in FP32 (~1 ulp); r = r^2 y0 refined by one Newton step in
//   FP64 (relative error ~1e-14; the FP64 form refines 1/r to FP64 first)
//   FP32C: r in wavelengths, phase = 2 pi fract(r), hardware sin/cos of turns;
//   FP64:  r in half wavelengths, phase = pi (q + t), q = rint(r), Taylor sin/cos
//   amplitude 1/r (FREESPACE) or r^{-3/2} (PNUSW) from y0; the remaining
//   constants are applied in FP64 in the finalize pass.
//
// Precision
//   FP32C: distance and phase reduction in FP64, sin/cos and amplitude in FP32,
//   FP32 MFMA partial sums flushed to FP64 every kFlushRounds rounds (256
//   elements per wave), FP64 across waves and items.
//   FP64: every step in FP64, FP64 MFMA accumulation.
//
// Determinism: every sum has a fixed order (waves in order through LDS, items
// of a drop in chunk order in the finalize pass), so results are bitwise
// repeatable regardless of which workgroup ran which item.
#include <mutex>

#include "device_math.h"
#include "internal.h"
#include "xlmimo.h"

namespace xl {

struct UserLane {
  double xp2;   // squared distance from the array line (ULA) or plane (UPA), (lambda/2) units
  double uy, uz;
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

// FP32C: distances are in units of lambda, so r counts whole turns of phase:
// h = a e^{-j 2 pi r} = a (cos(2 pi t) - j sin(2 pi t)),  t = fract(r) (v_fract_f64, exact),
// with the hardware v_sin_f32 / v_cos_f32, which take revolutions (measured on
// gfx950: |error| <= 1.3e-7 over a full turn).  Lanes with nothing to contribute
// (users beyond K, elements past the end) carry a coordinate of 1e30:
// rsq(inf) = 0 makes their entry exactly zero.
// Amplitude a (times us, a power of two: exact), c = cos(2 pi t) and sn = -sin(2 pi t),
// so that h = a (c + j sn).
template <int GEOM, int AMP>
__device__ __forceinline__ void channel_parts(double dy, double dz, double xp2, float us, float& a, float& c,
                                              float& sn) {
  double r2 = fma(dy, dy, xp2);
  if constexpr (GEOM == XLMIMO_UPA) r2 = fma(dz, dz, r2);
  const float yf = __builtin_amdgcn_rsqf((float)r2);
  const double y0 = (double)yf;
  const double r0 = r2 * y0;
  const double r = fma(0.5 * y0, fma(-r0, r0, r2), r0);
  const float t = (float)__builtin_amdgcn_fract(r);
  a = yf;
  if constexpr (AMP == XLMIMO_AMP_PNUSW) a = a * __builtin_amdgcn_sqrtf(a);
  a = a * us;
  c = __builtin_amdgcn_cosf(t);
  sn = __builtin_amdgcn_sinf(-t);
}

template <int GEOM, int AMP, bool SC = true>
__device__ __forceinline__ void channel_entry(double dy, double dz, double xp2, float& re, float& im) {
  float a, c, sn;
  channel_parts<GEOM, AMP>(dy, dz, xp2, 1.0f, a, c, sn);
  re = a * c;
  im = a * sn;
}

// FP64: distances in units of lambda / 2 (r counts half turns),
// h = a (-1)^q (cos(pi t) - j sin(pi t)), q = rint(r), t = r - q, Taylor sin/cos
// (SC: the series' coefficients in scalar registers).
template <int GEOM, int AMP, bool SC = true>
__device__ __forceinline__ void channel_entry(double dy, double dz, double xp2, double& re, double& im) {
  double r2 = fma(dy, dy, xp2);
  if constexpr (GEOM == XLMIMO_UPA) r2 = fma(dz, dz, r2);
  const double y = rsqrt_nr2(r2);  // 1 / r to FP64 rounding
  double r = r2 * y;
  r = fma(0.5 * y, fma(-r, r, r2), r);
  const double qd = __builtin_rint(r);
  double ns, c;
  sincos_half<SC>(r - qd, ns, c);
  double a = y;
  if constexpr (AMP == XLMIMO_AMP_PNUSW) a = a * sqrt(a);
  if (((int)qd) & 1) a = -a;
  re = a * c;
  im = a * ns;
}

// Squared distance of a user from the array line (ULA) or plane (UPA); the
// finalize pass recomputes it bit for bit for the split-half scales.
__device__ __forceinline__ double perp2(int geom, double x, double z) {
  return geom == XLMIMO_ULA ? fma(x, x, z * z) : x * x;
}

// Fixed-order sum of the 4 waves' partials through LDS, then one coalesced store.
template <int NV>
__device__ __forceinline__ void store_partial(const double* fin, double* s_red, double* __restrict__ part_out) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
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

// CROSS (NB == 4 only): a virtual drop of two 32-user groups of a larger drop,
// whose own blocks come from other virtual drops: only the products between
// user blocks {0, 1} and {2, 3} (16 MFMAs per round instead of 36); the other
// accumulators stay zero.
template <int NB, typename T, int GEOM, int AMP, bool CROSS = false>
__device__ void process_item(const ArrayK& arr, const DropK& dp, const ItemK& it, const double* __restrict__ pos,
                             double* __restrict__ part_out, double* s_red) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int NRE = NB * (NB + 1) / 2;
  constexpr int NX = NB * NB;
  constexpr int NV = (NRE + NX) * 4;
  constexpr bool F32 = sizeof(T) == 4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // metres -> wavelengths (FP32C, phase in turns) or half wavelengths (FP64, half turns)
  const double sc = (F32 ? 1.0 : 2.0) * arr.inv_lambda;
  constexpr double kFar = 1e30;            // coordinate of a lane that must contribute zero

  UserLane u[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int k = 16 * b + (lane & 15);
    double x = kFar, y = 0.0, z = 0.0;
    if (k < dp.k) {
      const double* p = pos + (dp.user_off + k) * 3;
      x = p[0] * sc;
      y = p[1] * sc;
      z = p[2] * sc;
    }
    u[b].xp2 = perp2(GEOM, x, z);
    u[b].uy = y;
    u[b].uz = z;
  }

  acc_t are[NRE], ax[NX];
#pragma unroll
  for (int i = 0; i < NRE; ++i) are[i] = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < NX; ++i) ax[i] = acc_t{0, 0, 0, 0};
  double carry[F32 ? NV : 1];
#pragma unroll
  for (int i = 0; i < (F32 ? NV : 1); ++i) carry[i] = 0.0;

  const int len = it.e_end - it.e_begin;
  const int n_full = len >> 4;                 // rounds with all 16 elements in range
  const int n_rounds = (len + 15) >> 4;
  const int e0 = it.e_begin + 4 * wave + (lane >> 4);
  const int ny = (GEOM == XLMIMO_ULA) ? dp.n_elems : arr.n_y;
  const double ds = arr.spacing * sc;
  const double cy = 0.5 * (double)(ny - 1) * ds;
  const double cz = 0.5 * (double)(arr.n_z - 1) * ds;

  static_assert(!CROSS || NB == 4, "cross-only items have two 32-user groups");
  auto round = [&](const double* dy, double ez) {
    T hre[NB], him[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) channel_entry<GEOM, AMP, (NB <= 2)>(dy[b], u[b].uz - ez, u[b].xp2, hre[b], him[b]);
    if constexpr (CROSS) {
      {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
          for (int bj = 2; bj < 4; ++bj) {
            const int t = tri_index(bi, bj, NB);
            are[t] = Mfma<T>::run(hre[bi], hre[bj], are[t]);
            are[t] = Mfma<T>::run(him[bi], him[bj], are[t]);
            ax[bi * NB + bj] = Mfma<T>::run(hre[bi], him[bj], ax[bi * NB + bj]);
            ax[bj * NB + bi] = Mfma<T>::run(hre[bj], him[bi], ax[bj * NB + bi]);
          }
        }
        return;
      }
    }
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
  };
  auto flush = [&]() {
    if constexpr (F32) {
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
  };

  // Blocks of kFlushRounds rounds: the element coordinate is recomputed exactly
  // at each block start.  FP32C advances y_user - y_element by 16 d per round
  // inside a block (<= 64 additions: < 1e-9 turns of error).
  for (int r0 = 0; r0 < n_rounds; r0 += kFlushRounds) {
    const int r1 = min(r0 + kFlushRounds, n_full);
    const int e = e0 + 16 * r0;
    double dy[NB];
    if constexpr (GEOM == XLMIMO_ULA) {
      const double ey = fma((double)e, ds, -cy);
#pragma unroll
      for (int b = 0; b < NB; ++b) dy[b] = u[b].uy - ey;
      if constexpr (F32) {
        const double step = 16.0 * ds;
        for (int r = r0; r < r1; ++r) {
          round(dy, 0.0);
#pragma unroll
          for (int b = 0; b < NB; ++b) dy[b] -= step;
        }
      } else {
        for (int r = r0; r < r1; ++r) {
          const double eyr = fma((double)(e + 16 * (r - r0)), ds, -cy);
#pragma unroll
          for (int b = 0; b < NB; ++b) dy[b] = u[b].uy - eyr;
          round(dy, 0.0);
        }
      }
    } else {
      int ea = e / arr.n_z, eb = e - (e / arr.n_z) * arr.n_z;
      for (int r = r0; r < r1; ++r) {
        const double eyr = fma((double)ea, ds, -cy);
#pragma unroll
        for (int b = 0; b < NB; ++b) dy[b] = u[b].uy - eyr;
        round(dy, fma((double)eb, ds, -cz));
        eb += 16;
        while (eb >= arr.n_z) {
          eb -= arr.n_z;
          ++ea;
        }
      }
    }
    if (r0 + kFlushRounds >= n_rounds && n_rounds > n_full) {
      // ragged last round: elements past the end take the far coordinate
      const int et = e0 + 16 * n_full;
      const bool valid = et < it.e_end;
      double ey, ez = 0.0;
      if constexpr (GEOM == XLMIMO_ULA) {
        ey = fma((double)et, ds, -cy);
      } else {
        const int ea = et / arr.n_z;
        ey = fma((double)ea, ds, -cy);
        ez = fma((double)(et - ea * arr.n_z), ds, -cz);
      }
      ey = valid ? ey : kFar;
#pragma unroll
      for (int b = 0; b < NB; ++b) dy[b] = u[b].uy - ey;
      round(dy, ez);
    }
    flush();
  }

  double fin[NV];
#pragma unroll
  for (int i = 0; i < NRE; ++i) {
#pragma unroll
    for (int c = 0; c < 4; ++c) fin[i * 4 + c] = F32 ? carry[i * 4 + c] : (double)are[i][c];
  }
#pragma unroll
  for (int i = 0; i < NX; ++i) {
#pragma unroll
    for (int c = 0; c < 4; ++c) fin[(NRE + i) * 4 + c] = F32 ? carry[(NRE + i) * 4 + c] : (double)ax[i][c];
  }

  store_partial<NV>(fin, s_red, part_out);
}

// ---------------------------------------------------------------------------
// FP32H: FP32C channel entries, products on the FP16 matrix cores.
//
// Each entry x (scaled per user by 2^q, a power of two chosen from the user's
// distance to the array so that |x| <= 1) is split as x = hi + lo with
// hi = f16(x), lo = f16(x - hi), both rounded to nearest; then
//   x_i x_j = hi_i hi_j + hi_i lo_j + lo_i hi_j + (lo_i lo_j, dropped)
// with |dropped| + rounding of lo <= ~2^-22 |x_i x_j| (or 2^-25 absolute where
// lo is subnormal), i.e. FP32-level products.  Three 16x16x32 FP16 MFMA per
// product stream cover 32 elements where FP32 MFMA needs eight.
// Work layout: a lane evaluates one user per 16-user block at a run of R
// consecutive elements, and 32 elements of each wave (one k-block of 8 per
// 16-lane group) feed one set of MFMAs: lane l holds row l % 16 and k-block l / 16
// of the 16x16x32 operands.  The per-element path takes R = 8 (one MFMA set per
// round, 128 elements per workgroup round); the expansion path takes R = 16 (its
// run feeds two MFMA sets, 256 elements per workgroup round).  Which element sits
// in which k slot does not matter as long as every user uses the same slots.
// Products accumulate in FP32 over 1024 elements per wave, then in FP64.
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
constexpr int kSplitFlushElems = 1024;   // elements per wave between FP64 carries
constexpr int kSplitMaxNb = 2;  // user blocks of 16 handled by the split kernel

__device__ __forceinline__ floatx4 mfma_h(halfx8 a, halfx8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Exponent q of the per-user scale 2^q: max over the array of |h| 2^q <= 1, from
// |h| <= xp2^{-1/2} (free space) or xp2^{-3/4} (PNUSW), xp2 the squared
// perpendicular distance in wavelengths.  Shared with the finalize pass.
__device__ __forceinline__ int split_exp(double xp2, int amp) {
  const int e = (xp2 > 0.0 && xp2 < 1e300) ? ilogb(xp2) : 0;
  const int q = amp == XLMIMO_AMP_FREESPACE ? (e >> 1) : ((3 * e) >> 2);
  return min(max(q, -100), 100);
}

// Entries m, m + 1 of the hi and lo operands from amplitudes a and c, sn (h = a (c + j sn)):
// hi = f16(a c) (two at a time: FP32 products, one packed conversion) and
// lo = f16(a c - hi) with a c exact inside the fused multiply-add, so
// hi + lo = a c to ~2^-22 relative.  lo is formed in FP32 (v_fma_mix_f32 reads
// hi straight from its FP16 half) and converted two at a time: on gfx950 the
// packed conversion and v_fma_mix_f32 issue like an FP32 FMA, while
// v_fma_mixlo_f16 / v_fma_mixhi_f16 (FP16 results into half registers) take
// over twice as long, so the empty asm statements keep the compiler from fusing
// the conversions into them (and make lo use these very hi values).
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_pair(const float* a, const float* c, const float* sn, halfx8& rh, halfx8& rl,
                                           halfx8& ih, halfx8& il, int m) {
  floatx2 pr = {a[0] * c[0], a[1] * c[1]};
  floatx2 pi = {a[0] * sn[0], a[1] * sn[1]};
  asm("" : "+v"(pr));
  asm("" : "+v"(pi));
  halfx2 hr = __builtin_convertvector(pr, halfx2);
  halfx2 hi = __builtin_convertvector(pi, halfx2);
  asm("" : "+v"(hr));
  asm("" : "+v"(hi));
  floatx2 lr = {__builtin_fmaf(a[0], c[0], -(float)hr[0]), __builtin_fmaf(a[1], c[1], -(float)hr[1])};
  floatx2 li = {__builtin_fmaf(a[0], sn[0], -(float)hi[0]), __builtin_fmaf(a[1], sn[1], -(float)hi[1])};
  asm("" : "+v"(lr));
  asm("" : "+v"(li));
  const halfx2 lrh = __builtin_convertvector(lr, halfx2);
  const halfx2 lih = __builtin_convertvector(li, halfx2);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    rh[m + q] = hr[q];
    ih[m + q] = hi[q];
    rl[m + q] = lrh[q];
    il[m + q] = lih[q];
  }
}

// Expansion of the channel along a lane's run of 16 consecutive elements (FP32H).
// The distance is exact in FP64 at the centre of the run (element m = 7.5, offset
// t = 0), its phase reduced there: c0 = fract(r_c).  Along the run the element
// offset is t = m' d, m' = m - 7.5, d the spacing in wavelengths, and with
// dy_c the centre's offset along the line, mu = dy_c / r_c:
//   r(t) - r_c = r_c sum_k C_k^(-1/2)(mu) (t / r_c)^k       (Gegenbauer generating function of
//   r(t)^-p    = r_c^-p sum_k C_k^(p/2)(mu) (t / r_c)^k      r_c^2 - 2 dy_c t + t^2)
// evaluated in FP32 by Horner's rule in m'^2 on the even and odd parts (the
// coefficients carry d^k), the phase to t^4 and the amplitude to t^3.  With the
// half-run |t| <= 7.5 d and every user at a distance x >= kExpandXmin d from the
// array line (plane), the truncated phase terms stay below 1e-7 turns (d <= 1);
// the first dropped amplitude term is at most C_4(1) (7.5 / 368)^4, 1.7e-7
// relative for free space and 4.3e-7 for the projected aperture (it peaks at the
// run's ends, where |m'| = 7.5).  The FP32 evaluation leaves |phase error| <=
// 5e-7 turns at d = 1/2 (9e-7 at d = 1: the phase is carried to |theta| < 4.3
// turns, so its rounding dominates) and 3e-7 relative in the amplitude.
// A second tier (TIER = 2) serves users between kExpandXmin2 = 184 and 368 spacings:
// the phase to t^6 (C_5 = mu (1 - mu^2)(7 mu^2 - 3) / 8, C_6 = (1 - mu^2)(21 mu^4
// - 14 mu^2 + 1) / 16) and the amplitude to t^4 (P_4, C_4^(3/4)); at x >= 184 d the
// first dropped phase term is below 5e-9 turns and the first dropped amplitude term
// at most C_5(1) (7.5 / 184)^5: 1.1e-7 (free space), 3.0e-7 (projected aperture).
// Three FMAs more per two elements.  Items whose users come closer still take the
// per-element FP64 path.
constexpr double kExpandXmin = 368.0;
constexpr double kExpandXmin2 = 184.0;
constexpr int kExpandRun = 16;

template <int AMP, int TIER = 1>
struct Expansion {
  float th[TIER == 2 ? 7 : 5];   // minus the phase in turns: -c0, then the coefficients of m', m'^2, ... (all negated)
  float am[TIER == 2 ? 5 : 4];   // amplitude (times the user scale): coefficients of 1, m', m'^2, ...
};

template <int AMP, int TIER = 1>
__device__ __forceinline__ Expansion<AMP, TIER> expand(double dyc, double xp2, double ds, float us) {
  Expansion<AMP, TIER> x;
  const double r2 = fma(dyc, dyc, xp2);
  const float yf = __builtin_amdgcn_rsqf((float)r2);
  const double y0 = (double)yf;
  const double r0 = r2 * y0;
  const double rc = fma(0.5 * y0, fma(-r0, r0, r2), r0);      // r_c to ~1e-14 relative
  const double y1 = fma(y0, fma(-rc, y0, 1.0), y0);           // 1 / r_c to ~1e-14 relative
  const double mu64 = dyc * y1;
  x.th[0] = -(float)__builtin_amdgcn_fract(rc);
  x.th[1] = (float)(mu64 * ds);
  const float mu = (float)mu64;
  const float dsf = (float)ds;
  const float q = yf * dsf;                                   // d / r_c
  const float w = __builtin_fmaf(-mu, mu, 1.0f);              // 1 - mu^2
  const float q2 = q * q;
  const float mu2 = mu * mu;
  const float qmu = q * mu;                                   // mu d / r_c, shared by three terms
  x.th[2] = (w * q) * (-0.5f * dsf);                          // -(1 - mu^2) d^2 / (2 r_c)
  x.th[3] = x.th[2] * qmu;                                    // -mu (1 - mu^2) d^3 / (2 r_c^2)
  x.th[4] = (x.th[2] * q2) * __builtin_fmaf(1.25f, mu2, -0.25f);   // -(1 - mu^2)(5 mu^2 - 1) d^4 / (8 r_c^3)
  float b0 = yf;
  if constexpr (AMP == XLMIMO_AMP_PNUSW) b0 = b0 * __builtin_amdgcn_sqrtf(b0);
  b0 = b0 * us;
  const float bq2 = b0 * q2;
  x.am[0] = b0;
  if constexpr (AMP == XLMIMO_AMP_FREESPACE) {          // Legendre polynomials P_k(mu)
    x.am[1] = b0 * qmu;
    x.am[2] = bq2 * __builtin_fmaf(1.5f, mu2, -0.5f);
    x.am[3] = bq2 * (qmu * __builtin_fmaf(2.5f, mu2, -1.5f));
  } else {                                              // C_k^(3/4)(mu)
    x.am[1] = b0 * (1.5f * qmu);
    x.am[2] = bq2 * __builtin_fmaf(2.625f, mu2, -0.75f);
    x.am[3] = bq2 * (qmu * __builtin_fmaf(4.8125f, mu2, -2.625f));
  }
  if constexpr (TIER == 2) {
    x.th[5] = (x.th[3] * q2) * __builtin_fmaf(1.75f, mu2, -0.75f);   // -mu (1 - mu^2)(7 mu^2 - 3) d^5 / (8 r_c^4)
    x.th[6] = (x.th[2] * (q2 * q2)) *
              __builtin_fmaf(__builtin_fmaf(2.625f, mu2, -1.75f), mu2, 0.125f);   // -C_6 d^6 / r_c^5
    if constexpr (AMP == XLMIMO_AMP_FREESPACE)
      x.am[4] = (bq2 * q2) * __builtin_fmaf(__builtin_fmaf(4.375f, mu2, -3.75f), mu2, 0.375f);
    else
      x.am[4] = (bq2 * q2) * __builtin_fmaf(__builtin_fmaf(9.0234375f, mu2, -7.21875f), mu2, 0.65625f);
  }
  return x;
}

// The two elements at m' = -p and +p from the even and odd parts of both series,
// with the phase carried negated (so that sn = sin(-theta) needs no sign flip):
// -theta(+-p) = E(p^2) +- p O(p^2), A(+-p) = Ae(p^2) +- p Ao(p^2) (9 FMAs per pair, 12 for
// the second tier).
template <int AMP, int TIER>
__device__ __forceinline__ void expansion_pair(const Expansion<AMP, TIER>& x, float p, float (&a)[2], float (&c)[2],
                                               float (&sn)[2]) {
  const float p2 = p * p;
  float ev, od, ae;
  if constexpr (TIER == 2) {
    ev = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(x.th[6], p2, x.th[4]), p2, x.th[2]), p2, x.th[0]);
    od = __builtin_fmaf(__builtin_fmaf(x.th[5], p2, x.th[3]), p2, x.th[1]);
    ae = __builtin_fmaf(__builtin_fmaf(x.am[4], p2, x.am[2]), p2, x.am[0]);
  } else {
    ev = __builtin_fmaf(__builtin_fmaf(x.th[4], p2, x.th[2]), p2, x.th[0]);
    od = __builtin_fmaf(x.th[3], p2, x.th[1]);
    ae = __builtin_fmaf(x.am[2], p2, x.am[0]);
  }
  const float ao = __builtin_fmaf(x.am[3], p2, x.am[1]);
  const float th0 = __builtin_fmaf(-p, od, ev), th1 = __builtin_fmaf(p, od, ev);
  a[0] = __builtin_fmaf(-p, ao, ae);
  a[1] = __builtin_fmaf(p, ao, ae);
  c[0] = __builtin_amdgcn_cosf(th0);
  sn[0] = __builtin_amdgcn_sinf(th0);
  c[1] = __builtin_amdgcn_cosf(th1);
  sn[1] = __builtin_amdgcn_sinf(th1);
}

// EXPAND: 0 the per-element FP64 path, 1 or 2 the expansion tier.
template <int NB, int GEOM, int AMP, int EXPAND>
__device__ void split_body(const ArrayK& arr, const DropK& dp, const ItemK& it, const UserLane (&u)[NB],
                           const float (&us)[NB], double* __restrict__ part_out, double* s_red);

// TIER2: whether users between 184 and 368 spacings take the second expansion tier (the kernels
// for batches of at most 32 users) or the per-element path (the kernels that also hold the larger
// drops' paths, whose register budget the second tier's code would strain).
template <int NB, int GEOM, int AMP, bool TIER2 = true>
__device__ void process_item_split(const ArrayK& arr, const DropK& dp, const ItemK& it,
                                   const double* __restrict__ pos, double* __restrict__ part_out, double* s_red) {
  const int lane = threadIdx.x & 63;
  const double sc = arr.inv_lambda;  // wavelengths: r counts turns
  constexpr double kFar = 1e30;
  UserLane u[NB];
  float us[NB];
  const double ds = arr.spacing * sc;
  const double xmin = kExpandXmin * ds, xmin2 = kExpandXmin2 * ds;
  bool near = false, near2 = false;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int k = 16 * b + (lane & 15);
    double x = kFar, y = 0.0, z = 0.0;
    if (k < dp.k) {
      const double* p = pos + (dp.user_off + k) * 3;
      x = p[0] * sc;
      y = p[1] * sc;
      z = p[2] * sc;
    }
    u[b].xp2 = perp2(GEOM, x, z);
    u[b].uy = y;
    u[b].uz = z;
    us[b] = k < dp.k ? __builtin_ldexpf(1.0f, split_exp(u[b].xp2, AMP)) : 1.0f;
    near |= !(u[b].xp2 >= xmin * xmin);
    near2 |= !(u[b].xp2 >= xmin2 * xmin2);
  }
  // every wave of the workgroup holds the same users, so they all take the same path
  const bool runs = GEOM == XLMIMO_ULA || arr.n_z % kExpandRun == 0;
  if (runs && !__any(near)) {
    split_body<NB, GEOM, AMP, 1>(arr, dp, it, u, us, part_out, s_red);
  } else if (TIER2 && runs && !__any(near2)) {
    if constexpr (TIER2) split_body<NB, GEOM, AMP, 2>(arr, dp, it, u, us, part_out, s_red);
  } else {
    split_body<NB, GEOM, AMP, 0>(arr, dp, it, u, us, part_out, s_red);
  }
}

template <int NB, int GEOM, int AMP, int EXPAND>
__device__ void split_body(const ArrayK& arr, const DropK& dp, const ItemK& it, const UserLane (&u)[NB],
                           const float (&us)[NB], double* __restrict__ part_out, double* s_red) {
  constexpr int NRE = NB * (NB + 1) / 2;
  constexpr int NX = NB * NB;
  constexpr int NV = (NRE + NX) * 4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const double sc = arr.inv_lambda;  // wavelengths: r counts turns
  constexpr double kFar = 1e30;

  floatx4 are[NRE], ax[NX];
#pragma unroll
  for (int i = 0; i < NRE; ++i) are[i] = floatx4{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < NX; ++i) ax[i] = floatx4{0, 0, 0, 0};
  double carry[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) carry[i] = 0.0;

  constexpr int RUN = EXPAND ? kExpandRun : 8;   // consecutive elements per lane and round
  constexpr int ROUND = 16 * RUN;                  // elements per workgroup round (4 waves x 4 groups)
  constexpr int FLUSH = kSplitFlushElems * 8 / (RUN * 32);   // rounds between FP64 carries
  const int len = it.e_end - it.e_begin;
  const int n_full = len / ROUND;
  const int n_rounds = (len + ROUND - 1) / ROUND;
  const int sub = RUN * (4 * wave + (lane >> 4));  // lane's first element within a round
  const int ny = (GEOM == XLMIMO_ULA) ? dp.n_elems : arr.n_y;
  const double ds = arr.spacing * sc;
  const double cy = 0.5 * (double)(ny - 1) * ds;
  const double cz = 0.5 * (double)(arr.n_z - 1) * ds;
  const int e0 = it.e_begin + sub;
  // The expansion path's run cursor, advanced by one round per call: on a line, every
  // user's offset from the run's centre (FP64, less one round's length per round); on a
  // plane, the column and row of the run's first element (runs never straddle a column).
  double dyc[NB];
  int ca = 0, cb = 0, qa = 0, qb = 0;
  if constexpr (EXPAND) {
    if constexpr (GEOM == XLMIMO_ULA) {
      const double ey0 = fma((double)e0 + 0.5 * (RUN - 1), ds, -cy);
#pragma unroll
      for (int b = 0; b < NB; ++b) dyc[b] = u[b].uy - ey0;
    } else {
      ca = e0 / arr.n_z;
      cb = e0 - ca * arr.n_z;
      qa = ROUND / arr.n_z;
      qb = ROUND - qa * arr.n_z;
    }
  }

  // One MFMA set: the 32 elements of each wave held as hi / lo operands.
  auto accumulate = [&](const halfx8 (&rh)[NB], const halfx8 (&rl)[NB], const halfx8 (&ih)[NB],
                        const halfx8 (&il)[NB]) {
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
      for (int bj = bi; bj < NB; ++bj) {
        floatx4& c = are[tri_index(bi, bj, NB)];
        c = mfma_h(rh[bi], rh[bj], c);
        c = mfma_h(ih[bi], ih[bj], c);
        c = mfma_h(rh[bi], rl[bj], c);
        c = mfma_h(ih[bi], il[bj], c);
        c = mfma_h(rl[bi], rh[bj], c);
        c = mfma_h(il[bi], ih[bj], c);
      }
    }
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
      for (int bj = 0; bj < NB; ++bj) {
        floatx4& c = ax[bi * NB + bj];
        c = mfma_h(rh[bi], ih[bj], c);
        c = mfma_h(rh[bi], il[bj], c);
        c = mfma_h(rl[bi], ih[bj], c);
      }
    }
  };

  // One round: the lane's RUN elements start at element index e; elements at or
  // past e_end (only in the last round, TAIL) contribute nothing.
  auto round = [&](int e, auto tail_tag) {
    constexpr bool TAIL = decltype(tail_tag)::value;
    if constexpr (EXPAND) {
      // the run's centre, element e + 7.5, and the expansion of each user about it
      Expansion<AMP, EXPAND> x[NB];
      if constexpr (GEOM == XLMIMO_ULA) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          x[b] = expand<AMP, EXPAND>(dyc[b], u[b].xp2, ds, us[b]);
          dyc[b] -= ROUND * ds;
        }
      } else {
        const double ey = fma((double)ca, ds, -cy);
        const double ez = fma((double)cb + 0.5 * (RUN - 1), ds, -cz);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double dy = u[b].uy - ey;
          x[b] = expand<AMP, EXPAND>(u[b].uz - ez, fma(dy, dy, u[b].xp2), ds, us[b]);
        }
        ca += qa;
        cb += qb;
        if (cb >= arr.n_z) {
          cb -= arr.n_z;
          ++ca;
        }
      }
      // set s takes the pairs m' = +-(4 s + j + 1/2), j = 0..3: operand slots 2j, 2j + 1
      // hold elements 7 - (4 s + j) and 8 + (4 s + j) of the run
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        halfx8 rh[NB], rl[NB], ih[NB], il[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int k = 4 * s + j;
            float a[2], c[2], sn[2];
            expansion_pair(x[b], 0.5f + (float)k, a, c, sn);
            if constexpr (TAIL) {
              a[0] = e + 7 - k < it.e_end ? a[0] : 0.0f;
              a[1] = e + 8 + k < it.e_end ? a[1] : 0.0f;
            }
            split_pair(a, c, sn, rh[b], rl[b], ih[b], il[b], 2 * j);
          }
        }
        accumulate(rh, rl, ih, il);
      }
    } else if constexpr (GEOM == XLMIMO_ULA) {
      halfx8 rh[NB], rl[NB], ih[NB], il[NB];
      const double ey = fma((double)e, ds, -cy);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        double dy = u[b].uy - ey;
#pragma unroll
        for (int m = 0; m < 8; m += 2) {
          float a[2], c[2], sn[2];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            double d = dy;
            dy -= ds;
            if constexpr (TAIL) d = e + m + q < it.e_end ? d : kFar;
            channel_parts<GEOM, AMP>(d, 0.0, u[b].xp2, us[b], a[q], c[q], sn[q]);
          }
          split_pair(a, c, sn, rh[b], rl[b], ih[b], il[b], m);
        }
      }
      accumulate(rh, rl, ih, il);
    } else {
      halfx8 rh[NB], rl[NB], ih[NB], il[NB];
      int ea = e / arr.n_z;
      int eb = e - ea * arr.n_z;
      float a[NB][2], c[NB][2], sn[NB][2];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        double ey = fma((double)ea, ds, -cy);
        const double ez = fma((double)eb, ds, -cz);
        if constexpr (TAIL) ey = e + m < it.e_end ? ey : kFar;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          channel_parts<GEOM, AMP>(u[b].uy - ey, u[b].uz - ez, u[b].xp2, us[b], a[b][m & 1], c[b][m & 1],
                                   sn[b][m & 1]);
        if (m & 1) {
#pragma unroll
          for (int b = 0; b < NB; ++b) split_pair(a[b], c[b], sn[b], rh[b], rl[b], ih[b], il[b], m - 1);
        }
        if (++eb == arr.n_z) {
          eb = 0;
          ++ea;
        }
      }
      accumulate(rh, rl, ih, il);
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < NRE; ++i) {
#pragma unroll
      for (int c = 0; c < 4; ++c) carry[i * 4 + c] += (double)are[i][c];
      are[i] = floatx4{0, 0, 0, 0};
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
      for (int c = 0; c < 4; ++c) carry[(NRE + i) * 4 + c] += (double)ax[i][c];
      ax[i] = floatx4{0, 0, 0, 0};
    }
  };

  for (int r0 = 0; r0 < n_full; r0 += FLUSH) {
    const int r1 = min(r0 + FLUSH, n_full);
    for (int r = r0; r < r1; ++r) round(e0 + ROUND * r, std::false_type{});
    flush();
  }
  if (n_rounds > n_full) {   // the partial last round, carried on its own
    round(e0 + ROUND * n_full, std::true_type{});
    flush();
  }
  store_partial<NV>(carry, s_red, part_out);
}

// ---------------------------------------------------------------------------
// FP32H for 64-user drops (four 16-user blocks).  The split operands of four blocks do not fit
// one lane beside the FP64 carries of all 26 accumulator blocks, so the work is divided by user
// block instead of by element: in every round all four waves take the same elements, wave w
// evaluates block w's users there (one user per lane, exactly as in the 16-user kernel), and
// publishes its hi / lo operands in LDS; after a barrier each wave forms its own share of the
// products — the cross blocks X[w, *] and two or three of the ten Re blocks — reading the other
// blocks' operands from LDS.  A lane then holds at most 7 accumulator blocks (and their
// carries), and each accumulator block lives in exactly one wave, which writes it to the
// partial image directly (the image layout of the other kernels, so the finalize pass is
// shared).  Re blocks per wave (bi <= bj), chosen so that every wave issues 24-30 MFMAs per set:
//   wave 0: (0,0) (0,1)   wave 1: (1,1) (1,2)   wave 2: (2,2) (2,3) (0,2)   wave 3: (3,3) (1,3) (0,3)
constexpr int kWideReN[4] = {2, 2, 3, 3};
constexpr int kWideRe[4][3][2] = {{{0, 0}, {0, 1}, {0, 0}},
                                  {{1, 1}, {1, 2}, {0, 0}},
                                  {{2, 2}, {2, 3}, {0, 2}},
                                  {{3, 3}, {1, 3}, {0, 3}}};

struct WideOps {
  halfx8 rh, rl, ih, il;
};

template <int W, int GEOM, int AMP, bool EXPAND>
__device__ void wide_body(const ArrayK& arr, const DropK& dp, const ItemK& it, const UserLane& u, float us,
                          double* __restrict__ part_out, double* s_red) {
  constexpr int NB = 4, NRE = 10;
  constexpr int NR = kWideReN[W];
  const int lane = threadIdx.x & 63;
  const double sc = arr.inv_lambda;
  constexpr double kFar = 1e30;
  constexpr int RUN = EXPAND ? kExpandRun : 8;   // consecutive elements per lane and round
  constexpr int SETS = RUN / 8;                  // 32-element MFMA sets per round
  constexpr int ROUND = 4 * RUN;                 // elements per round (all waves take the same ones)
  constexpr int FLUSH = kSplitFlushElems / (32 * SETS);   // rounds between FP64 carries
  // LDS operand exchange: [set][block][hi/lo array][lane], 16 bytes each
  halfx8* s_ops = reinterpret_cast<halfx8*>(s_red);
  auto ops_at = [&](int set, int b, int a) -> halfx8& { return s_ops[((set * NB + b) * 4 + a) * 64 + lane]; };

  floatx4 are[NR], ax[NB];
  double carry[(NR + NB) * 4];
#pragma unroll
  for (int i = 0; i < NR; ++i) are[i] = floatx4{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < NB; ++i) ax[i] = floatx4{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < (NR + NB) * 4; ++i) carry[i] = 0.0;

  const int len = it.e_end - it.e_begin;
  const int n_full = len / ROUND;
  const int n_rounds = (len + ROUND - 1) / ROUND;
  const int sub = RUN * (lane >> 4);
  const int ny = (GEOM == XLMIMO_ULA) ? dp.n_elems : arr.n_y;
  const double ds = arr.spacing * sc;
  const double cy = 0.5 * (double)(ny - 1) * ds;
  const double cz = 0.5 * (double)(arr.n_z - 1) * ds;
  const int e0 = it.e_begin + sub;
  // the expansion path's run cursor, advanced by one round per call (as in the 16-user kernel)
  double dyc = 0.0;
  int ca = 0, cb = 0, qa = 0, qb = 0;
  if constexpr (EXPAND) {
    if constexpr (GEOM == XLMIMO_ULA) {
      dyc = u.uy - fma((double)e0 + 0.5 * (RUN - 1), ds, -cy);
    } else {
      ca = e0 / arr.n_z;
      cb = e0 - ca * arr.n_z;
      qa = ROUND / arr.n_z;
      qb = ROUND - qa * arr.n_z;
    }
  }

  // own block's operands of one round (SETS sets), published to LDS
  auto evaluate = [&](int e, auto tail_tag) {
    constexpr bool TAIL = decltype(tail_tag)::value;
    if constexpr (EXPAND) {
      Expansion<AMP> x;
      if constexpr (GEOM == XLMIMO_ULA) {
        x = expand<AMP>(dyc, u.xp2, ds, us);
        dyc -= ROUND * ds;
      } else {
        const double ey = fma((double)ca, ds, -cy);
        const double ez = fma((double)cb + 0.5 * (RUN - 1), ds, -cz);
        const double dy = u.uy - ey;
        x = expand<AMP>(u.uz - ez, fma(dy, dy, u.xp2), ds, us);
        ca += qa;
        cb += qb;
        if (cb >= arr.n_z) {
          cb -= arr.n_z;
          ++ca;
        }
      }
#pragma unroll
      for (int s = 0; s < SETS; ++s) {
        WideOps o;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = 4 * s + j;
          float a[2], c[2], sn[2];
          expansion_pair<AMP>(x, 0.5f + (float)k, a, c, sn);
          if constexpr (TAIL) {
            a[0] = e + 7 - k < it.e_end ? a[0] : 0.0f;
            a[1] = e + 8 + k < it.e_end ? a[1] : 0.0f;
          }
          split_pair(a, c, sn, o.rh, o.rl, o.ih, o.il, 2 * j);
        }
        ops_at(s, W, 0) = o.rh;
        ops_at(s, W, 1) = o.rl;
        ops_at(s, W, 2) = o.ih;
        ops_at(s, W, 3) = o.il;
      }
    } else if constexpr (GEOM == XLMIMO_ULA) {
      WideOps o;
      const double ey = fma((double)e, ds, -cy);
      double dy = u.uy - ey;
#pragma unroll
      for (int m = 0; m < 8; m += 2) {
        float a[2], c[2], sn[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          double d = dy;
          dy -= ds;
          if constexpr (TAIL) d = e + m + q < it.e_end ? d : kFar;
          channel_parts<GEOM, AMP>(d, 0.0, u.xp2, us, a[q], c[q], sn[q]);
        }
        split_pair(a, c, sn, o.rh, o.rl, o.ih, o.il, m);
      }
      ops_at(0, W, 0) = o.rh;
      ops_at(0, W, 1) = o.rl;
      ops_at(0, W, 2) = o.ih;
      ops_at(0, W, 3) = o.il;
    } else {
      WideOps o;
      int ea = e / arr.n_z;
      int eb = e - ea * arr.n_z;
      float a[2], c[2], sn[2];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        double ey = fma((double)ea, ds, -cy);
        const double ez = fma((double)eb, ds, -cz);
        if constexpr (TAIL) ey = e + m < it.e_end ? ey : kFar;
        channel_parts<GEOM, AMP>(u.uy - ey, u.uz - ez, u.xp2, us, a[m & 1], c[m & 1], sn[m & 1]);
        if (m & 1) split_pair(a, c, sn, o.rh, o.rl, o.ih, o.il, m - 1);
        if (++eb == arr.n_z) {
          eb = 0;
          ++ea;
        }
      }
      ops_at(0, W, 0) = o.rh;
      ops_at(0, W, 1) = o.rl;
      ops_at(0, W, 2) = o.ih;
      ops_at(0, W, 3) = o.il;
    }
  };

  // this wave's products of one round, from the four blocks' operands in LDS
  auto contract = [&]() {
#pragma unroll
    for (int s = 0; s < SETS; ++s) {
      WideOps b[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        b[k].rh = ops_at(s, k, 0);
        b[k].rl = ops_at(s, k, 1);
        b[k].ih = ops_at(s, k, 2);
        b[k].il = ops_at(s, k, 3);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int bi = kWideRe[W][r][0], bj = kWideRe[W][r][1];
        floatx4& c = are[r];
        c = mfma_h(b[bi].rh, b[bj].rh, c);
        c = mfma_h(b[bi].ih, b[bj].ih, c);
        c = mfma_h(b[bi].rh, b[bj].rl, c);
        c = mfma_h(b[bi].ih, b[bj].il, c);
        c = mfma_h(b[bi].rl, b[bj].rh, c);
        c = mfma_h(b[bi].il, b[bj].ih, c);
      }
#pragma unroll
      for (int bj = 0; bj < NB; ++bj) {
        floatx4& c = ax[bj];
        c = mfma_h(b[W].rh, b[bj].ih, c);
        c = mfma_h(b[W].rh, b[bj].il, c);
        c = mfma_h(b[W].rl, b[bj].ih, c);
      }
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
#pragma unroll
      for (int c = 0; c < 4; ++c) carry[i * 4 + c] += (double)are[i][c];
      are[i] = floatx4{0, 0, 0, 0};
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
#pragma unroll
      for (int c = 0; c < 4; ++c) carry[(NR + i) * 4 + c] += (double)ax[i][c];
      ax[i] = floatx4{0, 0, 0, 0};
    }
  };

  for (int r0 = 0; r0 < n_full; r0 += FLUSH) {
    const int r1 = min(r0 + FLUSH, n_full);
    for (int r = r0; r < r1; ++r) {
      evaluate(e0 + ROUND * r, std::false_type{});
      __syncthreads();   // every block's operands of this round are in LDS
      contract();
      __syncthreads();   // every wave has read them before the next round overwrites them
    }
    flush();
  }
  if (n_rounds > n_full) {   // the partial last round, carried on its own
    evaluate(e0 + ROUND * n_full, std::true_type{});
    __syncthreads();
    contract();
    __syncthreads();
    flush();
  }
  // each accumulator block lives in this wave alone: straight into the partial image
  // (value v = block * 4 + register at v * 64 + lane; Re blocks by tri_index, then X blocks)
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int blk = tri_index(kWideRe[W][r][0], kWideRe[W][r][1], NB);
#pragma unroll
    for (int c = 0; c < 4; ++c) part_out[(blk * 4 + c) * 64 + lane] = carry[r * 4 + c];
  }
#pragma unroll
  for (int bj = 0; bj < NB; ++bj) {
    const int blk = NRE + W * NB + bj;
#pragma unroll
    for (int c = 0; c < 4; ++c) part_out[(blk * 4 + c) * 64 + lane] = carry[(NR + bj) * 4 + c];
  }
  __syncthreads();   // the LDS exchange buffer is free again for the next item
}

template <int GEOM, int AMP>
__device__ void process_item_wide(const ArrayK& arr, const DropK& dp, const ItemK& it,
                                  const double* __restrict__ pos, double* __restrict__ part_out, double* s_red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double sc = arr.inv_lambda;
  constexpr double kFar = 1e30;
  const double ds = arr.spacing * sc;
  const double xmin = kExpandXmin * ds;
  // this wave's user: block `wave`
  const int k = 16 * wave + (lane & 15);
  double x = kFar, y = 0.0, z = 0.0;
  if (k < dp.k) {
    const double* p = pos + (dp.user_off + k) * 3;
    x = p[0] * sc;
    y = p[1] * sc;
    z = p[2] * sc;
  }
  UserLane u;
  u.xp2 = perp2(GEOM, x, z);
  u.uy = y;
  u.uz = z;
  const float us = k < dp.k ? __builtin_ldexpf(1.0f, split_exp(u.xp2, AMP)) : 1.0f;
  // the expansion's condition over all 64 users of the workgroup (the waves hold different ones)
  __shared__ int s_near;
  if (threadIdx.x == 0) s_near = 0;
  __syncthreads();
  if (__any(!(u.xp2 >= xmin * xmin)) && lane == 0) atomicOr(&s_near, 1);
  __syncthreads();
  const bool expand = (GEOM == XLMIMO_ULA || arr.n_z % kExpandRun == 0) && s_near == 0;
  switch (wave) {
    case 0: expand ? wide_body<0, GEOM, AMP, true>(arr, dp, it, u, us, part_out, s_red)
                   : wide_body<0, GEOM, AMP, false>(arr, dp, it, u, us, part_out, s_red); break;
    case 1: expand ? wide_body<1, GEOM, AMP, true>(arr, dp, it, u, us, part_out, s_red)
                   : wide_body<1, GEOM, AMP, false>(arr, dp, it, u, us, part_out, s_red); break;
    case 2: expand ? wide_body<2, GEOM, AMP, true>(arr, dp, it, u, us, part_out, s_red)
                   : wide_body<2, GEOM, AMP, false>(arr, dp, it, u, us, part_out, s_red); break;
    default: expand ? wide_body<3, GEOM, AMP, true>(arr, dp, it, u, us, part_out, s_red)
                    : wide_body<3, GEOM, AMP, false>(arr, dp, it, u, us, part_out, s_red); break;
  }
}

template <int NBMAX, typename T, int GEOM, int AMP, bool SPLIT>
__global__ __launch_bounds__(kGramThreads) __attribute__((amdgpu_waves_per_eu(SPLIT && NBMAX <= 2 ? 4 / NBMAX : (NBMAX == kNbWide ? 2 : 1)))) void k_gram_exact(ArrayK arr, const DropK* __restrict__ drops,
                                                               const double* __restrict__ pos,
                                                               const ItemK* __restrict__ items, int n_items,
                                                               int* __restrict__ counter,
                                                               double* __restrict__ partials,
                                                               const int32_t* __restrict__ mask,
                                                               const int* __restrict__ n_items_dev) {
  constexpr bool WIDE_ONLY = NBMAX == kNbWide;   // no 3-block or cross-group drop in the batch
  constexpr int NBM = WIDE_ONLY ? 4 : NBMAX;
  __shared__ double s_red[partial_values(NBM) * 64];
  __shared__ int s_item;
  if (n_items_dev != nullptr) n_items = *n_items_dev;   // a compacted item list: its length is on the device
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = s_item;
    __syncthreads();
    if (idx >= n_items) break;  // uniform over the workgroup: every wave leaves together
    const ItemK it = items[idx];
    if (mask != nullptr && mask[it.drop] == 0) continue;  // drop not selected: skip its items
    const DropK dp = drops[it.drop];
    double* out = partials + dp.part_off + it.chunk * (int64_t)(partial_values(dp.nb) * 64);
    if constexpr (SPLIT) {
      switch (dp.nb) {
        case 1: process_item_split<1, GEOM, AMP, (NBM <= 2)>(arr, dp, it, pos, out, s_red); break;
        case 2: if constexpr (NBM >= 2) process_item_split<2, GEOM, AMP, (NBM <= 2)>(arr, dp, it, pos, out, s_red); break;
        // 33-48 users, and the cross blocks of virtual drops (more than 64 users): FP32C products
        case 3: if constexpr (NBM >= 3 && !WIDE_ONLY) process_item<3, float, GEOM, AMP>(arr, dp, it, pos, out, s_red); break;
        case 4:
          if constexpr (WIDE_ONLY) {
            process_item_wide<GEOM, AMP>(arr, dp, it, pos, out, s_red);
          } else if constexpr (NBM >= 4) {
            if (dp.cross) process_item<4, float, GEOM, AMP, true>(arr, dp, it, pos, out, s_red);
            else process_item_wide<GEOM, AMP>(arr, dp, it, pos, out, s_red);
          }
          break;
        default: break;
      }
    } else {
      switch (dp.nb) {
        case 1: process_item<1, T, GEOM, AMP>(arr, dp, it, pos, out, s_red); break;
        case 2: if constexpr (NBM >= 2) process_item<2, T, GEOM, AMP>(arr, dp, it, pos, out, s_red); break;
        case 3: if constexpr (NBM >= 3) process_item<3, T, GEOM, AMP>(arr, dp, it, pos, out, s_red); break;
        case 4:
          if constexpr (NBM >= 4) {
            if (dp.cross) process_item<4, T, GEOM, AMP, true>(arr, dp, it, pos, out, s_red);
            else process_item<4, T, GEOM, AMP>(arr, dp, it, pos, out, s_red);
          }
          break;
        default: break;
      }
    }
  }
}

__global__ void k_reset_counter(int* counter) {
  if (threadIdx.x == 0) *counter = 0;
}

// The work items of the selected drops: one thread per item and one slot range per wave (an
// atomic on the count, which k_reset_counter zeroes first).  The list's order follows the waves'
// atomics; it decides only which workgroup takes which item, since every item writes its own
// partial image and the finalize pass sums a drop's images in chunk order.
__global__ __launch_bounds__(256) void k_compact_items(const ItemK* __restrict__ items, int n_items,
                                                       const int32_t* __restrict__ mask, ItemK* __restrict__ out,
                                                       int* __restrict__ count) {
  const int i = blockIdx.x * 256 + threadIdx.x, lane = threadIdx.x & 63;
  ItemK it{};
  bool keep = false;
  if (i < n_items) {
    it = items[i];
    keep = mask[it.drop] != 0;
  }
  const unsigned long long bal = __ballot(keep);
  int base = 0;
  if (lane == 0 && bal != 0ull) base = atomicAdd(count, __popcll(bal));
  base = __shfl(base, 0, 64);
  if (keep) out[base + __popcll(bal & ((1ull << lane) - 1ull))] = it;
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
                                                       double* __restrict__ gram,
                                                       const int32_t* __restrict__ mask, int split) {
  if (mask != nullptr && mask[blockIdx.x] == 0) return;
  const DropK dp = drops[blockIdx.x];
  const int K = dp.k, NB = dp.nb;
  const int NRE = NB * (NB + 1) / 2;
  const int64_t PV = partial_values(NB) * 64;
  const double* base = partials + dp.part_off;
  constexpr double kPi = 3.14159265358979323846264338327950288;
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
    // Lanes carried 1/r' (or r'^{-3/2}) with r' = su r, su = 1/lambda (FP32C) or 2/lambda (FP64).
    const double su = (sizeof(T) == 4 ? 1.0 : 2.0) * arr.inv_lambda;
    double scale;
    if (arr.amp == XLMIMO_AMP_FREESPACE) {
      const double c = arr.lambda * su / (4.0 * kPi);  // (lambda / 4 pi)^2 su^2
      scale = c * c;
    } else {
      const double* up = pos + (dp.user_off + p) * 3;
      const double* uq = pos + (dp.user_off + q) * 3;
      const double xp = (arr.geom == XLMIMO_ULA) ? sqrt(fma(up[0], up[0], up[2] * up[2])) : fabs(up[0]);
      const double xq = (arr.geom == XLMIMO_ULA) ? sqrt(fma(uq[0], uq[0], uq[2] * uq[2])) : fabs(uq[0]);
      scale = arr.beta0 * sqrt(xp * xq) * su * su * su;
    }
    if (split && (NB <= kSplitMaxNb || (NB == 4 && !dp.cross))) {
      // undo the per-user scales 2^q of the split-half entries (exact powers of two)
      const double* up = pos + (dp.user_off + p) * 3;
      const double* uq = pos + (dp.user_off + q) * 3;
      const int qp = split_exp(perp2(arr.geom, up[0] * su, up[2] * su), arr.amp);
      const int qq = split_exp(perp2(arr.geom, uq[0] * su, uq[2] * su), arr.amp);
      scale = ldexp(scale, -(qp + qq));
    }
    if (i > j) im = -im;  // G_ji = conj(G_ij)
    gram[(dp.gram_off + idx) * 2] = re * scale;
    gram[(dp.gram_off + idx) * 2 + 1] = im * scale;
  }
}

template <int NBMAX, typename T, int GEOM, int AMP, bool SPLIT>
static int occupancy_grid() {
  static int cached = 0;
  if (!cached) {
    int dev = 0, n_cu = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gram_exact<NBMAX, T, GEOM, AMP, SPLIT>, kGramThreads, 0);
    cached = (n_cu > 0 ? n_cu : 256) * (per_cu > 0 ? per_cu : 1);
  }
  return cached;
}

template <typename T, int GEOM, int AMP, bool SPLIT>
static int grid_nb(int nb_max) {
  if constexpr (SPLIT) {
    if (nb_max == kNbWide) return occupancy_grid<kNbWide, T, GEOM, AMP, SPLIT>();
  }
  return nb_max <= 1 ? occupancy_grid<1, T, GEOM, AMP, SPLIT>()
                     : (nb_max <= 2 ? occupancy_grid<2, T, GEOM, AMP, SPLIT>() : occupancy_grid<4, T, GEOM, AMP, SPLIT>());
}

template <typename T, bool SPLIT>
static int grid_t(int nb_max, int geom, int amp) {
  if (geom == XLMIMO_ULA)
    return amp == XLMIMO_AMP_FREESPACE ? grid_nb<T, XLMIMO_ULA, XLMIMO_AMP_FREESPACE, SPLIT>(nb_max)
                                       : grid_nb<T, XLMIMO_ULA, XLMIMO_AMP_PNUSW, SPLIT>(nb_max);
  return amp == XLMIMO_AMP_FREESPACE ? grid_nb<T, XLMIMO_UPA, XLMIMO_AMP_FREESPACE, SPLIT>(nb_max)
                                     : grid_nb<T, XLMIMO_UPA, XLMIMO_AMP_PNUSW, SPLIT>(nb_max);
}

int gram_exact_grid(int precision, int nb_max, int geom, int amp) {
  if (precision == XLMIMO_FP64) return grid_t<double, false>(nb_max, geom, amp);
  if (precision == XLMIMO_FP32H) return grid_t<float, true>(nb_max, geom, amp);
  return grid_t<float, false>(nb_max, geom, amp);
}

struct MainArgs {
  ArrayK arr;
  const DropK* drops;
  const double* pos;
  const ItemK* items;
  int n_items;
  int* counter;
  double* partials;
  const int32_t* mask;
  const int* n_items_dev;
};

template <typename T, int GEOM, int AMP, bool SPLIT>
static void launch_main(int nb_max, int grid, hipStream_t s, const MainArgs& a) {
  if constexpr (SPLIT) {
    if (nb_max == kNbWide) {
      k_gram_exact<kNbWide, T, GEOM, AMP, SPLIT><<<grid, kGramThreads, 0, s>>>(a.arr, a.drops, a.pos, a.items, a.n_items, a.counter, a.partials, a.mask, a.n_items_dev);
      return;
    }
  }
  if (nb_max <= 1)
    k_gram_exact<1, T, GEOM, AMP, SPLIT><<<grid, kGramThreads, 0, s>>>(a.arr, a.drops, a.pos, a.items, a.n_items, a.counter, a.partials, a.mask, a.n_items_dev);
  else if (nb_max <= 2)
    k_gram_exact<2, T, GEOM, AMP, SPLIT><<<grid, kGramThreads, 0, s>>>(a.arr, a.drops, a.pos, a.items, a.n_items, a.counter, a.partials, a.mask, a.n_items_dev);
  else
    k_gram_exact<4, T, GEOM, AMP, SPLIT><<<grid, kGramThreads, 0, s>>>(a.arr, a.drops, a.pos, a.items, a.n_items, a.counter, a.partials, a.mask, a.n_items_dev);
}

template <typename T, bool SPLIT>
static void launch_t(int nb_max, int grid, hipStream_t s, const MainArgs& a) {
  if (a.arr.geom == XLMIMO_ULA) {
    if (a.arr.amp == XLMIMO_AMP_FREESPACE) launch_main<T, XLMIMO_ULA, XLMIMO_AMP_FREESPACE, SPLIT>(nb_max, grid, s, a);
    else launch_main<T, XLMIMO_ULA, XLMIMO_AMP_PNUSW, SPLIT>(nb_max, grid, s, a);
  } else {
    if (a.arr.amp == XLMIMO_AMP_FREESPACE) launch_main<T, XLMIMO_UPA, XLMIMO_AMP_FREESPACE, SPLIT>(nb_max, grid, s, a);
    else launch_main<T, XLMIMO_UPA, XLMIMO_AMP_PNUSW, SPLIT>(nb_max, grid, s, a);
  }
}

hipError_t launch_gram_exact(int precision, int nb_max, const ArrayK& arr, const DropK* d_drops, int n_drops,
                             const double* d_pos, const ItemK* d_items, int n_items, int* d_counter,
                             double* d_partials, double* d_gram, int grid, hipStream_t s, hipEvent_t ev0,
                             hipEvent_t ev1, const int32_t* d_mask, ItemK* d_items_sel, int* d_n_sel) {
  if (n_drops == 0) return hipSuccess;
  k_reset_counter<<<1, 64, 0, s>>>(d_counter);
  if (grid < 1) grid = 1;
  MainArgs a{arr, d_drops, d_pos, d_items, n_items, d_counter, d_partials, d_mask, nullptr};
  if (d_mask != nullptr && d_items_sel != nullptr && d_n_sel != nullptr) {
    // a few selected drops: pop only their items
    k_reset_counter<<<1, 64, 0, s>>>(d_n_sel);
    if (n_items > 0) k_compact_items<<<(n_items + 255) / 256, 256, 0, s>>>(d_items, n_items, d_mask, d_items_sel, d_n_sel);
    a.items = d_items_sel;
    a.n_items_dev = d_n_sel;
  }
  if (ev0) (void)hipEventRecord(ev0, s);
  if (precision == XLMIMO_FP64) launch_t<double, false>(nb_max, grid, s, a);
  else if (precision == XLMIMO_FP32H) launch_t<float, true>(nb_max, grid, s, a);
  else launch_t<float, false>(nb_max, grid, s, a);
  if (ev1) (void)hipEventRecord(ev1, s);
  if (precision == XLMIMO_FP64)
    k_gram_finalize<double><<<n_drops, 256, 0, s>>>(arr, d_drops, d_pos, d_partials, d_gram, d_mask, 0);
  else
    k_gram_finalize<float><<<n_drops, 256, 0, s>>>(arr, d_drops, d_pos, d_partials, d_gram, d_mask,
                                                   precision == XLMIMO_FP32H);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free exact Gram (xlmimo_gram_exact_noalloc): its
// queue counter, launch plan and per-item partial sums, in one file-scope
// device array that each GPU holds from the module's load to the end of the
// process.  Host code never names the array itself (its host-side name is a
// stand-in, not a device address): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// every launch and copy uses that address.
static __device__ __align__(256) unsigned char scratch[XLMIMO_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;   // the caller makes the device current
  void* ptr = nullptr;
  e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace xl
