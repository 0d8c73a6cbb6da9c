// Virtual drops of the exact Gram: the fused kernel of gram_exact.hip sees at
// most 64 users per work item, so larger drops (and the rows of moved users)
// run as virtual drops whose positions are gathered first and whose Grams are
// scattered back into the callers' K x K outputs.
#include "internal.h"

namespace xl {

// Drops with more users than one work item holds run as virtual drops, one per
// pair of user groups: their positions are gathered in virtual-user order
// first, and every virtual Gram's blocks are copied into the real drop's K x K
// output after (the virtual Grams are already full Hermitian).
__global__ __launch_bounds__(256) void k_gather_users(const double* __restrict__ pos, const int64_t* __restrict__ map,
                                                      int64_t n_vusers, double* __restrict__ vpos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_vusers * 3) return;
  const int64_t u = t / 3;
  vpos[t] = pos[map[u] * 3 + (t - u * 3)];
}

// One workgroup per virtual drop; entry (r, c) of its (ka + kb)^2 Gram is
// copied when it lies in the cross blocks or in a group's own block that the
// descriptor assigns to this virtual drop.
__global__ __launch_bounds__(256) void k_scatter_groups(const VDropK* __restrict__ vd,
                                                        const double2* __restrict__ vgram,
                                                        double2* __restrict__ gram) {
  const VDropK v = vd[blockIdx.x];
  const int kv = v.ka + v.kb;
  for (int idx = threadIdx.x; idx < kv * kv; idx += blockDim.x) {
    const int r = idx / kv, c = idx - (idx / kv) * kv;
    const bool ra = r < v.ka, ca = c < v.ka;
    if (ra && ca && !(v.flags & kVCopyA)) continue;
    if (!ra && !ca && !(v.flags & kVCopyB)) continue;
    const int gr = ra ? v.a0 + r : v.b0 + (r - v.ka);
    const int gc = ca ? v.a0 + c : v.b0 + (c - v.ka);
    gram[v.gram_off + (int64_t)gr * v.k + gc] = vgram[v.vgram_off + idx];
  }
}

// Row update: one workgroup per virtual drop; row 0 and column 0 of its Gram
// (the moved user against its partners) land in row m and column m.
__global__ __launch_bounds__(256) void k_scatter_rows(const VRowK* __restrict__ vr, const int64_t* __restrict__ map,
                                                      const double2* __restrict__ vgram,
                                                      double2* __restrict__ gram) {
  const VRowK v = vr[blockIdx.x];
  const int m = (int)(map[v.vu0] - v.user_off);
  for (int c = threadIdx.x; c < v.kv; c += blockDim.x) {
    if (c == 0) {
      if (v.diag) gram[v.gram_off + (int64_t)m * v.k + m] = vgram[v.vgram_off];
      continue;
    }
    const int j = (int)(map[v.vu0 + c] - v.user_off);
    gram[v.gram_off + (int64_t)m * v.k + j] = vgram[v.vgram_off + c];
    gram[v.gram_off + (int64_t)j * v.k + m] = vgram[v.vgram_off + (int64_t)c * v.kv];
  }
}

hipError_t launch_scatter_rows(const VRowK* d_vr, int n_vr, const int64_t* d_map, const double* d_vgram,
                               double* d_gram, hipStream_t s) {
  if (n_vr == 0) return hipSuccess;
  k_scatter_rows<<<n_vr, 256, 0, s>>>(d_vr, d_map, reinterpret_cast<const double2*>(d_vgram),
                                      reinterpret_cast<double2*>(d_gram));
  return hipGetLastError();
}

hipError_t launch_gather_users(const double* d_pos, const int64_t* d_map, int64_t n_vusers, double* d_vpos,
                               hipStream_t s) {
  if (n_vusers == 0) return hipSuccess;
  const int64_t n = n_vusers * 3;
  k_gather_users<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d_pos, d_map, n_vusers, d_vpos);
  return hipGetLastError();
}

hipError_t launch_scatter_groups(const VDropK* d_v, int n_v, const double* d_vgram, double* d_gram, hipStream_t s) {
  if (n_v == 0) return hipSuccess;
  k_scatter_groups<<<n_v, 256, 0, s>>>(d_v, reinterpret_cast<const double2*>(d_vgram),
                                       reinterpret_cast<double2*>(d_gram));
  return hipGetLastError();
}

}  // namespace xl
