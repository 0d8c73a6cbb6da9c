// Internal declarations shared by the C-ABI layer and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xl {

// Array description as the kernels see it.
struct ArrayK {
  int32_t geom;       // XLMIMO_ULA / XLMIMO_UPA
  int32_t amp;        // XLMIMO_AMP_*
  int32_t n_y, n_z;   // UPA panel (ULA: per-drop N in DropK)
  double spacing;
  double lambda;
  double inv_lambda;
  double beta0;
};

// One drop of a batch, device resident.
// Gauss-Legendre nodes of the closed forms' Fresnel integrals F(s), |s| <= 8
// (at most 32 rad of phase over [0, s]); the table follows the 64-node rule.
constexpr int kFresnelNodes = 32;

struct DropK {
  int64_t user_off;   // first user in the position array
  int64_t gram_off;   // first complex element of the drop's K x K output
  int64_t part_off;   // first double of the drop's partials (exact Gram)
  int64_t pair_off;   // first user pair (i < j) of the drop in pair-indexed buffers
  int32_t n_elems;    // antennas (ULA: N, UPA: n_y * n_z)
  int32_t k;          // users
  int32_t nb;         // ceil(k / 16) user blocks
  int32_t n_items;    // work items (element chunks) of this drop
  int32_t cross;      // virtual drop of two 32-user groups whose own blocks come from elsewhere:
                      // only the products between user blocks {0, 1} and {2, 3}
  int32_t pad_;
};

// One work item of the exact Gram: a contiguous element range of one drop.
struct ItemK {
  int32_t drop;
  int32_t chunk;      // partial = drops[drop].part_off + chunk * partial_values(nb) * 64
  int32_t e_begin;
  int32_t e_end;
};

// A drop with more users than one work item holds (K > XLMIMO_MAX_USERS) runs
// as virtual drops: its users fall in groups of kGroupUsers (the last one
// shorter), and every pair of groups (a < b) is one virtual drop with group a's
// users (user blocks 0-1) then group b's (blocks 2-3).  One descriptor per
// virtual drop tells the scatter which blocks of the virtual Gram land where in
// the real one.
constexpr int kGroupUsers = 32;
enum : int32_t { kVCopyA = 1, kVCopyB = 2 };   // also copy group a's / b's own block
struct VDropK {
  int64_t gram_off;   // the real drop's first complex element
  int64_t vgram_off;  // the virtual drop's first complex element in the virtual Gram
  int32_t k;          // the real drop's K
  int32_t a0, ka;     // group a: first user (drop-local) and size
  int32_t b0, kb;     // group b
  int32_t flags;      // kVCopyA | kVCopyB; the cross block a-b is always copied
};

// Row update of moved users: virtual drop = one moved user m (virtual user 0)
// and up to 63 partner users of its drop; only row 0 and column 0 of its Gram
// are copied back, into row m and column m of the real drop.
struct VRowK {
  int64_t gram_off;   // the real drop's first complex element
  int64_t vgram_off;  // the virtual drop's first complex element in the virtual Gram
  int64_t user_off;   // the real drop's first user (global index)
  int64_t vu0;        // the virtual drop's first virtual user (into the user map)
  int32_t k;          // the real drop's K
  int32_t kv;         // users of the virtual drop (1 + partners)
  int32_t diag;       // also copy G_mm (the first virtual drop of each moved user)
  int32_t pad;
};

// Values of one partial: per lane, NB(NB+1)/2 symmetric Re blocks and NB^2
// cross blocks, 4 accumulator registers each.
__host__ __device__ constexpr int partial_values(int nb) { return (nb * (nb + 1) / 2 + nb * nb) * 4; }
__host__ __device__ constexpr int tri_index(int bi, int bj, int nb) {
  // index of block (bi <= bj) in row-major upper-triangular order
  return bi * nb - bi * (bi - 1) / 2 + (bj - bi);
}

constexpr int kGramThreads = 256;     // 4 waves per work item
// Plan-level user-block bound of the exact Gram's launch: 1, 2 or 4 (the largest drop's
// 16-user blocks), or kNbWide for batches whose largest drops have four blocks while no drop
// has three and none is a cross-group virtual drop (the FP32H launch then runs a kernel without
// the FP32C paths those need, at half the registers).
constexpr int kNbWide = 5;
constexpr int kFlushRounds = 64;      // FP32 MFMA partial sums are carried to FP64 every 64 rounds (256 elements per wave)

// BF16 GEMM for the learned correction (mlp.hip): C[M x N] = sum_k A(m,k) B(k,n),
// A(m,k) = A[m a_m + k a_k], B(k,n) = B[k b_k + n b_n], outputs row-major with pitch ldo.
enum { EPI_FWD_HIDDEN = 0, EPI_FWD_OUT = 1, EPI_BWD_DX = 2, EPI_STORE_F32 = 3 };
struct GemmArgs {
  int M, N, K;
  const __bf16* A;
  int64_t a_m, a_k;
  const __bf16* B;
  int64_t b_k, b_n;
  const float* bias;  // [N]: FWD_HIDDEN, FWD_OUT
  float* Z;           // FWD_HIDDEN: pre-activations out (may be null); BWD_DX: pre-activations in
  __bf16* out_bf;     // FWD_HIDDEN: GELU(z); BWD_DX: dZ of the previous layer
  float* out_f;       // FWD_OUT, STORE_F32 (split-K: [splits][M][ldo] partials)
  int64_t ldo;
  int k_chunk;        // STORE_F32 split-K: K range per grid.z slice (0 = whole K)
  int row_sums;       // STORE_F32: also write sum_k A(m, k) after the M x ldo block of each slice
};

// Launchers (stream-ordered, no host synchronisation).
hipError_t launch_gram_exact(int precision, int nb_max, const ArrayK& arr, const DropK* d_drops, int n_drops,
                             const double* d_pos, const ItemK* d_items, int n_items, int* d_counter,
                             double* d_partials, double* d_gram, int grid, hipStream_t s, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr, const int32_t* d_mask = nullptr,
                             ItemK* d_items_sel = nullptr, int* d_n_sel = nullptr);
int gram_exact_grid(int precision, int nb_max, int geom, int amp);
// Virtual drops: positions gathered by user map, blocks scattered back.
hipError_t launch_gather_users(const double* d_pos, const int64_t* d_map, int64_t n_vusers, double* d_vpos,
                               hipStream_t s);
hipError_t launch_scatter_groups(const VDropK* d_v, int n_v, const double* d_vgram, double* d_gram, hipStream_t s);
hipError_t launch_scatter_rows(const VRowK* d_vr, int n_vr, const int64_t* d_map, const double* d_vgram,
                               double* d_gram, hipStream_t s);

hipError_t launch_closedform(const ArrayK& arr, const DropK* d_drops, int n_drops, int variant, const double* d_pos,
                             const double* d_gl, int n_gl, double* d_diag, double* d_gram, int32_t* d_status,
                             int k_max, hipStream_t s, int64_t n_pairs = 0,
                             int32_t* d_route = nullptr);

// k_max > XLMIMO_MAX_USERS runs the workgroup-per-drop kernel, whose matrices
// live in d_work (complex128, one K x K block per drop at its Gram offset).
hipError_t launch_rates(const DropK* d_drops, int n_drops, int k_max, const double* d_gram, const double* d_filter,
                        int n_snr, const double* d_rho, int64_t total_users, int schemes, double* d_rates,
                        int32_t* d_status, hipStream_t s, double* d_work = nullptr);

// Cholesky factors for tracking (LAPACK column-major L at each drop's Gram offset).
hipError_t launch_cholesky(const DropK* d_drops, int n_drops, const double* d_gram, const double* d_rho,
                           double* d_factor, double* d_logdet, int32_t* d_status, hipStream_t s);
hipError_t launch_chol_update(const DropK* d_drops, int n_mdrops, const int32_t* d_mdrop, const int32_t* d_moff,
                              const int32_t* d_mloc, const double* d_gram, const double* d_rho, double* d_factor,
                              double* d_logdet, int32_t* d_status, hipStream_t s);

hipError_t launch_ergodic(const double* d_rates, int n_drops, int n_vals, double* d_out, hipStream_t s);
hipError_t launch_y_bounds(const double* d_pos, const DropK* d_drops, int n_drops, int geom, double t_sat,
                           double* d_bounds, hipStream_t s);
hipError_t launch_saturation(const double* d_bounds, int n_drops, const double* d_ergodic, const double* d_nlist,
                             int n_N, int n_vals, double spacing, double eps, double* d_sat, hipStream_t s);

hipError_t launch_gemm(int epi, const GemmArgs& g, hipStream_t s);
hipError_t launch_pair_inputs(const ArrayK& arr, const DropK* d_drops, int n_drops, const double* d_pos,
                              const double* d_cf, const double* d_exact, __bf16* feat, float* aux, float* target,
                              int32_t* pmap, hipStream_t s);
// loss == nullptr: the per-block partial sums are left for launch_adam_layers.
hipError_t launch_mlp_head(int64_t n, const float* out, const float* aux, const float* target, __bf16* dout,
                           double* partial, double* loss, hipStream_t s);
// Split-K GEMM into out[M x ldo] (fixed-order sum over the slices); with row_sums, also
// out[M * ldo + m] = sum_k A(m, k) (the bias gradient of a weight-gradient GEMM).
hipError_t launch_gemm_splitk(const GemmArgs& g, int splits, float* partial, float* out, hipStream_t s);
// Split-K weight-gradient GEMM that leaves its slices unreduced: partial[z][M * ldo (+ M)];
// returns the number of slices actually used through *slices.
hipError_t launch_gemm_splitk_partials(const GemmArgs& g, int splits, float* partial, int* slices, hipStream_t s);
// The unreduced slices of every layer's weight and bias gradients: layer l owns parameters
// [start[l], start[l + 1]) and its slices sit at part + part_off[l] + z (start[l + 1] - start[l]).
constexpr int kMaxLayers = 17;
struct SplitLayers {
  int32_t n;
  int32_t splits[kMaxLayers];
  int32_t in_dim[kMaxLayers];   // layer l: in_dim[l] inputs, (start[l + 1] - start[l]) / (in_dim[l] + 1) outputs
  int64_t start[kMaxLayers + 1];
  int64_t part_off[kMaxLayers];
};
// Split-K GEMMs (EPI_STORE_F32, unreduced slices into partials[p]) of up to kMaxLayers
// problems in one launch; all problems must share the operands' fetch modes (else
// hipErrorInvalidValue).  slices[p] returns the slices used by problem p.
struct GemmGroup {
  int32_t n;
  int32_t first[kMaxLayers + 1];
  int32_t gx[kMaxLayers], gy[kMaxLayers];
  GemmArgs g[kMaxLayers];
};
hipError_t launch_gemm_grouped_partials(const GemmArgs* gs, const int* splits, float* const* partials, int n,
                                       int* slices, hipStream_t s);
// grad[i] = sum over slices (in slice order) of parameter i's partials.
hipError_t launch_reduce_layers(const SplitLayers& L, const float* part, float* grad, hipStream_t s);
// Adam on every parameter, with the gradient summed from the slices as launch_reduce_layers does
// (bitwise the same gradient), or read from grad when part == nullptr; the BF16 copy wbf and
// its per-layer transpose wbf_t (layer l's weights as [in][out] at start[l]) follow.  With
// loss != nullptr, block 0 also sums the loss head's per-block partials into
// *loss = sum / n_pairs (the order of launch_mlp_head's sum).
hipError_t launch_adam_layers(const SplitLayers& L, const float* part, const float* grad, int64_t n, float* w,
                              float* m, float* v, float lr, float b1, float b2, float eps, float bc1, float bc2,
                              __bf16* wbf, __bf16* wbf_t, const double* loss_part, int n_loss_part, int64_t n_pairs,
                              double* loss, hipStream_t s);
// wbf_t = per-layer transpose of the weights in w (BF16), layers as in L (start, in_dim).
hipError_t launch_weights_t(const SplitLayers& L, const float* w, __bf16* wbf_t, hipStream_t s);
hipError_t launch_to_bf16(int64_t n, const float* w, __bf16* wbf, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_or_flags(int32_t* status, const int32_t* flags, int64_t n, int32_t bit, hipStream_t s);
// Fallback gate of the learned correction: a drop falls back to the exact Gram
// when a pair's predicted log-variance exceeds min(cap, thr[b]), b the first bin
// with N <= n_upper[b] (no bin: cap alone).
constexpr int kGateBins = 16;
struct GateK {
  int32_t n_bins;
  float cap;
  int64_t n_upper[kGateBins];
  float thr[kGateBins];
};
hipError_t launch_mlp_apply(int64_t n, const float* out, const float* aux, const int32_t* pmap, const DropK* d_drops,
                            double* gram, int32_t* flags, const GateK& gate, hipStream_t s);
hipError_t launch_mlp_fused_forward(int width, int depth, int64_t n, const __bf16* feat, const __bf16* wbf,
                                    const float* master, const int64_t* d_offs, float* out, hipStream_t s);
// What the training forward keeps for the backward pass: hidden layer l's pre-activation
// z[l] (FP32, n x width) and its GELU output x[l + 1] (BF16, n x width, the next layer's input).
struct FwdKeep {
  float* z[kMaxLayers];
  __bf16* x[kMaxLayers];
};
// The fused forward of the training step (widths 64, 128, 256): the inference kernel's pass,
// storing keep.z / keep.x of every hidden layer besides the output.  Returns
// hipErrorInvalidValue for other widths (the caller runs the layer GEMMs instead).
hipError_t launch_mlp_fused_train_forward(int width, int depth, int64_t n, const __bf16* feat, const __bf16* wbf,
                                          const float* master, const int64_t* d_offs, const FwdKeep& keep,
                                          float* out, hipStream_t s);
// The input-gradient chain of the training step in one fused pass (widths 64, 128, 256): from the
// output gradient dout (BF16, n x 8) down through every layer, dZ[l - 1] = (dZ[l] W[l]) * GELU'(z[l - 1]),
// stored to dz[l - 1] (BF16, n x width) for the weight gradients; W[l]^T is read from wbf_t.
struct BwdKeep {
  const float* z[kMaxLayers];
  __bf16* dz[kMaxLayers];
};
hipError_t launch_mlp_fused_train_backward(int width, int depth, int64_t n, const __bf16* dout, const __bf16* wbf_t,
                                           const int64_t* d_offs, const BwdKeep& keep, hipStream_t s);
constexpr int kMlpHeadBlocks = 256;
constexpr int kDoutPitch = 8;   // bf16 per pair of the output-layer gradient (7 used; 16-byte rows)

// Allocation-free exact Gram: the per-device address of the static scratch
// array (XLMIMO_NOALLOC_SCRATCH_BYTES).  static_scratch_init looks it up once
// per device, with that device current; static_scratch returns it (nullptr
// before the look-up).
hipError_t static_scratch_init(int device);
void* static_scratch(int device);

}  // namespace xl
