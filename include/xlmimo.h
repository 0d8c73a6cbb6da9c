/*
 * xlmimo.h - C ABI of the MI355X (gfx950) library for near-field XL-MIMO
 * multiuser Gram matrices, linear-receiver sum-rates and capacity saturation,
 * and their updates as users move (tracking).
 *
 * Method: Cui, Park, Alouini, "Channel Capacity Saturation Point and
 * Beamforming Acceleration for Near-Field XL-MIMO Multiuser Communications".
 *
 * Conventions shared by every entry point
 *   - Units are SI (metres); SNRs are linear, never dB.
 *   - Complex numbers are interleaved (re, im) pairs of double.
 *   - Pointers documented as DEVICE must point to memory of the context's
 *     device (hipMalloc'd or a torch tensor's data_ptr()); HOST pointers are
 *     ordinary process memory read before the call returns.  The caller owns
 *     all of them; the library allocates only its own workspace, held by the
 *     context.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *     is asynchronous: outputs are valid once the stream has synchronised.
 *   - Return codes: XLMIMO_OK, or a negative whole-call error.  Whole-call
 *     errors are detected on the host before anything is enqueued
 *     (XLMIMO_EINVAL) or come from the HIP runtime (XLMIMO_EDEVICE, text in
 *     xlmimo_last_error).  Per-drop numerical conditions never fail a call:
 *     they are reported in per-drop status words (XLMIMO_ST_* bits).
 *   - Calls on one context are serialised by an internal mutex, and they
 *     share the context's workspace: work enqueued by two calls of one
 *     context on different streams must not overlap in time (use one context
 *     per stream for concurrent work).
 *   - The first call with a new batch shape builds and uploads a launch plan
 *     synchronously; later calls with the same shape enqueue kernels only, so
 *     a warmed-up call sequence can be captured into a hipGraph
 *     (xlmimo_graph_begin / xlmimo_graph_end below).
 */
#ifndef XLMIMO_H
#define XLMIMO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XLMIMO_OK        0
#define XLMIMO_EINVAL   (-1)   /* invalid argument (message in xlmimo_last_error) */
#define XLMIMO_EDEVICE  (-2)   /* HIP runtime error */
#define XLMIMO_ENOMEM   (-3)   /* workspace allocation failed */
#define XLMIMO_ENOTIMPL (-4)   /* combination not implemented */

/* Array geometry (Sec. II-A: the ULA lies on the y axis, centred at the
 * origin; the UPA is the same construction in the y-z plane).
 * ULA element n = 0..N-1 sits at (0, (n - (N-1)/2) d, 0); UPA element
 * (a, b) sits at (0, (a - (n_y-1)/2) d, (b - (n_z-1)/2) d). */
#define XLMIMO_ULA 0
#define XLMIMO_UPA 1

/* Channel amplitude model.
 * FREESPACE: h = lambda / (4 pi r) e^{-j 2 pi r / lambda}.
 * PNUSW (eq. (3)): h = sqrt(beta0) e^{-j 2 pi r / lambda} / r * sqrt(x_perp / r),
 *   x_perp = distance of the user from the array line (ULA) or plane (UPA). */
#define XLMIMO_AMP_FREESPACE 0
#define XLMIMO_AMP_PNUSW     1

/* Exact-Gram precision.
 * FP64 : distance, phase, sin/cos, amplitude and accumulation in FP64.
 * FP32C: distance and phase reduction (2 pi r / lambda modulo 2 pi) in FP64,
 *        sin/cos and amplitude in FP32, products summed in FP32 over blocks
 *        of at most 256 elements whose partial sums are carried in FP64. */
#define XLMIMO_FP64  0
#define XLMIMO_FP32C 1
/* FP32H: FP32C entries, each scaled per user by a power of two (|x| <= 1) and
 *        split as hi + lo (FP16 each, rounded to nearest); products hi hi +
 *        hi lo + lo hi on the FP16 matrix cores with FP32 accumulation, carried
 *        in FP64 as for FP32C.  Each product is exact to ~2^-22 relative
 *        (FP32 level); users need x_perp >= 2^-100 wavelengths. */
#define XLMIMO_FP32H 2

/* Closed-form variants (eqs. (4), (6), (22), (23); see xlmimo_gram_closedform). */
#define XLMIMO_CF_PAPER 0      /* formulas as printed, for every pair */
#define XLMIMO_CF_GATED 1      /* off-diagonal set to 0 when the stationary point is off the aperture */
/* The next two are ULA-only extensions beyond the paper's formulas.  Some pairs
 * are evaluated numerically: "slow-phase" pairs, for which k |u_i - u_j| times
 * the angle the aperture subtends at the pair's midpoint is at most 960 rad
 * (users a fraction of a metre apart: no stationary-phase regime), and pairs
 * whose stationary zone is broad (Fresnel width >= 1/2 of the half-aperture: the
 * phase is far from quadratic over it) when that costs at most N/8 quadrature
 * nodes.  Their entry is the aperture integral (1/d) int conj(h_i) h_j dy by
 * composite Gauss-Legendre quadrature plus the discrete end corrections, or the
 * direct sum over the N elements when N <= 1024 or that costs no more. */
#define XLMIMO_CF_UNIFORM 2    /* uniform stationary-phase form of the discrete sum: the stationary term
                                  weighted by the Fresnel integral between the array ends, end terms
                                  without their stationary singularity, discrete end corrections;
                                  numeric pairs as above */
#define XLMIMO_CF_GATED_QUAD 3 /* GATED, numeric pairs as above (the learned correction's base) */

/* Rate schemes (bitmask).  rates_out holds one value per set bit, in
 * increasing bit order. */
#define XLMIMO_ZF         1    /* sum log2(1 + rho_k / [G^-1]_kk) */
#define XLMIMO_MMSE       2    /* sum log2(1 / [(I + D^1/2 G D^1/2)^-1]_kk) */
#define XLMIMO_MRC        4    /* sum log2(1 + rho_k G_kk^2 / (sum_{j!=k} rho_j |G_kj|^2 + G_kk)) */
#define XLMIMO_CAP        8    /* log2 det(I + D^1/2 G D^1/2), eq. (9) */
#define XLMIMO_MZF       16    /* ZF formula evaluated on the filter Gram (nominal modified ZF) */
#define XLMIMO_MZF_MISM  32    /* modified-ZF filter G~^-1 H^H applied to the true channel */
#define XLMIMO_CORR_GAP  64    /* not a rate: -(1/K) log2 det R, R_ij = G_ij / sqrt(G_ii G_jj), the largest
                                  normalised gap between the Hadamard and Schur-Horn capacity bounds
                                  (Appendix A, eq. (9)); the same value at every SNR */

/* Per-drop status bits. */
#define XLMIMO_ST_G_NOT_PD      1   /* Cholesky of the ZF Gram failed: ZF-type rates are NaN */
#define XLMIMO_ST_MMSE_NOT_PD   2   /* Cholesky of I + A failed: MMSE/CAP are NaN */
#define XLMIMO_ST_FILTER_NOT_PD 4   /* Cholesky of the filter Gram failed: XLMIMO_MZF is NaN;
                                       XLMIMO_MZF_MISM then inverts G~ by Gauss-Jordan with partial
                                       pivoting (NaN only if G~ is singular) */
#define XLMIMO_ST_BAD_INPUT     8   /* non-finite position or a user on the array line/plane */
#define XLMIMO_ST_CF_DEGENERATE 16  /* closed form hit |x_i| == |x_j| or coincident users (entry set to 0) */
#define XLMIMO_ST_FELL_BACK     32  /* learned correction was uncertain: the drop's Gram was computed exactly */

/* Capacity-sweep Gram forms. */
#define XLMIMO_FORM_EXACT_FP64  0
#define XLMIMO_FORM_EXACT_FP32C 1
#define XLMIMO_FORM_CF_PAPER    2
#define XLMIMO_FORM_CF_GATED    3
#define XLMIMO_FORM_CF_GATED_MLP 4  /* gated closed form + learned residual + exact fallback */
#define XLMIMO_FORM_EXACT_FP32H 5   /* exact Gram at XLMIMO_FP32H precision */
#define XLMIMO_FORM_CF_UNIFORM  6   /* closed form, variant XLMIMO_CF_UNIFORM */

/* Users per drop: at most XLMIMO_MAX_USERS for the closed forms and the learned
 * form; the exact Gram, the sum-rates (all schemes but XLMIMO_MZF and
 * XLMIMO_MZF_MISM) and the exact capacity sweeps take up to
 * XLMIMO_MAX_USERS_EXACT (the Appendix A study runs to K = 1000). */
#define XLMIMO_MAX_USERS 64
#define XLMIMO_MAX_USERS_EXACT 1024

/* Learned correction: network inputs and outputs per user pair. */
#define XLMIMO_MLP_IN  6
#define XLMIMO_MLP_OUT 7
#define XLMIMO_PAIR_FEAT_PITCH 8   /* bf16 features per pair (6 used) */
#define XLMIMO_PAIR_AUX_PITCH  8   /* floats per pair: 3 complex phasors, sqrt(G~_ii G~_jj), pad */

typedef struct xlmimo_ctx xlmimo_ctx;
typedef struct xlmimo_mlp xlmimo_mlp;

/* Receive array and channel model. */
typedef struct {
  int32_t geometry;      /* XLMIMO_ULA or XLMIMO_UPA */
  int32_t amp_model;     /* XLMIMO_AMP_FREESPACE or XLMIMO_AMP_PNUSW */
  int64_t n_y, n_z;      /* ULA: n_y = default N, n_z = 1. UPA: panel size */
  double  spacing_m;     /* element spacing d > 0 (the paper uses lambda / 2) */
  double  wavelength_m;  /* lambda > 0 */
  double  beta0;         /* PNUSW gain constant (the paper sets 1); ignored for FREESPACE */
} xlmimo_array;

/* A batch of Monte-Carlo drops, possibly uneven in N and K. */
typedef struct {
  int64_t        n_drops;  /* >= 0; 0 makes every call a no-op */
  const int64_t* n_elems;  /* HOST [n_drops]: ULA antennas per drop; NULL = array n_y. Ignored for UPA */
  const int32_t* n_users;  /* HOST [n_drops]: users per drop, 1..XLMIMO_MAX_USERS (_EXACT, see above) */
  const double*  user_pos; /* DEVICE [total_users][3]: x, y, z of each user, drops back to back */
} xlmimo_batch;

/* Output layout of every Gram: drop d's K_d x K_d complex matrix, row-major,
 * full Hermitian, starts at complex element sum_{d' < d} K_{d'}^2. */

int         xlmimo_ctx_create(xlmimo_ctx** out, int device);
int         xlmimo_ctx_destroy(xlmimo_ctx* ctx);
const char* xlmimo_last_error(const xlmimo_ctx* ctx);
const char* xlmimo_version(void);

/* Benchmark timing of the exact-Gram main kernel (not part of the method).
 * While enabled, every exact-Gram launch of this context (also those made by
 * xlmimo_capacity_sweep) is bracketed by a pair of hipEvents recorded on its
 * launch stream.  xlmimo_timing_read waits for the recorded events, returns
 * the summed kernel time in ms and the number of launches, and clears the
 * record.  Events are created on demand and reused; enabling or disabling
 * clears the record. */
int xlmimo_timing_enable(xlmimo_ctx* ctx, int on);
int xlmimo_timing_read(xlmimo_ctx* ctx, double* total_ms, int64_t* n_launches);

/* Exact Gram G = H^H H (Sec. III: G_ii = P_i / P, rho_ij = G_ij / sqrt(G_ii G_jj);
 * Sec. V-B: the inner products the paper accelerates).  H is generated on the
 * fly from the geometry and user positions and never stored.
 *   precision  XLMIMO_FP64, XLMIMO_FP32C or XLMIMO_FP32H
 *   gram_out   DEVICE complex128, layout above
 * Drops with a non-finite position or a user at distance 0 from an element
 * get NaN entries (no status array here; xlmimo_zf_mmse_sumrate flags them).
 * K up to XLMIMO_MAX_USERS_EXACT.  A drop with K > XLMIMO_MAX_USERS is split
 * into groups of 32 users (the last one shorter) and every pair of groups
 * runs as one work item of at most 64 users: pairs of neighbouring groups
 * compute their whole Gram (and give each group its own block), the others
 * only the products between their two groups; the blocks are then copied
 * into the drop's K x K output.  Workspace grows with the sum over such drops
 * of (groups choose 2) x 64^2 complex values plus the per-item partial sums. */
int xlmimo_gram_exact(xlmimo_ctx* ctx, const xlmimo_array* arr, const xlmimo_batch* batch,
                      int32_t precision, double* gram_out, void* stream);

/* Allocation-free exact Gram, for callers that cannot allocate device memory
 * during the call (tight serving loops, harnesses that forbid hipMalloc after
 * start-up).  It computes what xlmimo_gram_exact computes, with
 * the same kernels, and calls no hipMalloc, hipFree or other allocating
 * routine: its queue counter, launch plan and per-item partial sums live in
 * one static device array of XLMIMO_NOALLOC_SCRATCH_BYTES per GPU, held from
 * the library's first use of that GPU until the process ends; its address is
 * taken once per device by xlmimo_ctx_create.
 *   ctx        a context of the GPU to run on (device, error text); none of
 *              its workspace is used
 *   arr, batch, precision, gram_out  as in xlmimo_gram_exact
 *   stream     as in xlmimo_gram_exact
 * Limits: K <= XLMIMO_MAX_USERS per drop, and the batch's plan and partial
 * sums must fit the static array (56 B per drop, plus 16 B and
 * (nb(nb+1)/2 + nb^2) x 2 KiB per work item, nb = ceil(K/16); work items are
 * element ranges of the length xlmimo_gram_exact picks for the batch,
 * lengthened up to one item per drop when needed).  A batch beyond them
 * returns XLMIMO_EINVAL before anything is enqueued.  Untuned, the work items
 * equal those of xlmimo_gram_exact, and the Grams are bit-identical to its
 * own.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (the queue counter is cleared by a kernel at the start of each call):
 * calls whose work overlaps in time on one GPU race, whatever their context
 * or stream.  Each call uploads its launch plan with an asynchronous copy on
 * `stream` from a static host buffer (pageable memory, so the call is not
 * meant for graph capture); a call first waits until the previous call's
 * upload has completed. */
#define XLMIMO_NOALLOC_SCRATCH_BYTES (64u << 20)
int xlmimo_gram_exact_noalloc(xlmimo_ctx* ctx, const xlmimo_array* arr, const xlmimo_batch* batch,
                              int32_t precision, double* gram_out, void* stream);

/* Tracking update of the exact Gram (Sec. V-B: user states known from sensing
 * let the channel be regenerated as users move).  After users of the batch
 * have moved (their new positions already written to batch->user_pos),
 * recompute the rows and columns of gram_inout that involve them; every other
 * entry is left as it is.  Replacing row and column m of G is a Hermitian
 * rank-2 change.  Each moved user m runs as work items of itself and at most
 * 63 other users of its drop, so a row costs about K channel evaluations per
 * element against the full Gram's K (K <= 64) or (ceil(K/32) - 1) K (K > 64).
 *   precision   XLMIMO_FP64, XLMIMO_FP32C or XLMIMO_FP32H (as xlmimo_gram_exact)
 *   moved       HOST int64 [n_moved]: global user indices (drops back to back),
 *               strictly ascending; an entry between two moved users is written
 *               by the row of the lower index
 *   gram_inout  DEVICE complex128 Grams (layout above) of the previous positions
 * K up to XLMIMO_MAX_USERS_EXACT.  A new moved set builds a launch plan
 * synchronously (warm it before graph capture); the context keeps the plans
 * of the last 16 moved sets, apart from its other plans. */
int xlmimo_gram_update_users(xlmimo_ctx* ctx, const xlmimo_array* arr, const xlmimo_batch* batch,
                             int32_t precision, int64_t n_moved, const int64_t* moved, double* gram_inout,
                             void* stream);

/* Cholesky factors for tracking.  The factored matrix of a drop is its Gram G
 * (rho == NULL) or I + D^1/2 G D^1/2 with D = diag(rho) for one SNR (the MMSE /
 * capacity matrix).  The factor L (A = L L^H, real positive diagonal) is FP64
 * complex in LAPACK column-major order: element (i, j), i >= j, at complex
 * element gram_off + j K + i of the Gram layout above, the strict upper
 * triangle zero.  log2 det A = 2 sum_k log2 L_kk gives the capacity
 * log2 det(I + A) directly (eq. (9)).
 *   gram        DEVICE complex128 Grams (layout above)
 *   rho         DEVICE double [total_users] or NULL
 *   factor_out  DEVICE complex128, the Gram's size
 *   logdet_out  DEVICE double [n_drops] or NULL: log2 det A (NaN when not PD)
 *   status_out  DEVICE int32 [n_drops] or NULL: 0, or XLMIMO_ST_G_NOT_PD
 *               (XLMIMO_ST_MMSE_NOT_PD with rho) with the factor undefined
 * One 512-thread workgroup per drop, K up to XLMIMO_MAX_USERS_EXACT. */
int xlmimo_cholesky(xlmimo_ctx* ctx, const xlmimo_batch* batch, const double* gram, const double* rho,
                    double* factor_out, double* logdet_out, int32_t* status_out, void* stream);

/* Tracking update of the factors: after xlmimo_gram_update_users has replaced
 * the rows and columns of the moved users in `gram`, bring factors made by
 * xlmimo_cholesky (same rho) up to date.  Per moved user m the change of A is
 * Hermitian rank 2, u e_m^H + e_m u^H (u: the new column m minus the old one,
 * the old one from L L^H, u_m halved) = v1 v1^H - v2 v2^H with
 * v1,2 = (u / s +- s e_m) / sqrt 2; one pass over the columns applies the
 * rotation of the rank-1 update with v1 and the hyperbolic rotation of the
 * downdate with v2: O(K^2) per moved user against O(K^3) for a new
 * factorisation.  Moved users of a drop are applied in ascending order.
 *   arr, batch, moved  as in xlmimo_gram_update_users (they share its cached plan)
 *   logdet_out, status_out  as in xlmimo_cholesky, written only for drops with
 *               moved users; a downdate that meets a non-positive pivot (A no
 *               longer positive definite) sets the status bit, and the factor
 *               is then undefined: factor the matrix anew.
 * Repeated updates accumulate rounding; refactor from time to time. */
int xlmimo_cholesky_update_users(xlmimo_ctx* ctx, const xlmimo_array* arr, const xlmimo_batch* batch,
                                 int64_t n_moved, const int64_t* moved, const double* gram, const double* rho,
                                 double* factor_inout, double* logdet_out, int32_t* status_out, void* stream);

/* Closed-form Gram of the paper's modified ZF (eqs. (22)-(23)):
 *   G~_ii = eq. (4) / P (PNUSW ULA, general spacing d: beta0/(d x_i) S_i with
 *           half-aperture L = N d / 2); the free-space ULA analogue
 *           (lambda/4pi)^2 /(d x_i) [atan((L-y_i)/x_i) + atan((L+y_i)/x_i)];
 *           the UPA panel integral of |h|^2 / d^2.
 *   G~_ij = rho_ij sqrt(G~_ii G~_jj) with rho_ij of eq. (6) (sgn of eq. (7)),
 *           or the corresponding stationary-phase term for the free-space
 *           ULA and the UPA (phase offset -pi/2 on the panel).
 *   variant     XLMIMO_CF_PAPER or XLMIMO_CF_GATED; for a ULA also XLMIMO_CF_UNIFORM
 *               or XLMIMO_CF_GATED_QUAD (see their definitions; not the paper's formulas)
 *   gram_out    DEVICE complex128, layout above
 *   status_out  DEVICE int32 [n_drops] or NULL: XLMIMO_ST_BAD_INPUT,
 *               XLMIMO_ST_CF_DEGENERATE bits (overwritten, not or-ed). */
int xlmimo_gram_closedform(xlmimo_ctx* ctx, const xlmimo_array* arr, const xlmimo_batch* batch,
                           int32_t variant, double* gram_out, int32_t* status_out, void* stream);

/* ZF / MMSE / MRC / capacity / modified-ZF sum-rates of every drop (eq. (9),
 * eq. (21) and the textbook linear-receiver SINRs), from batched FP64
 * Cholesky factorisations of K x K Grams.
 *   gram_true    DEVICE complex128 Grams (layout above)
 *   gram_filter  DEVICE complex128 Grams used by XLMIMO_MZF / XLMIMO_MZF_MISM; may be NULL otherwise
 *   n_snr        number of SNR points (>= 1)
 *   rho          DEVICE double [n_snr][total_users]: rho_k = P_k / sigma^2 (linear)
 *   schemes      bitmask of XLMIMO_ZF ... XLMIMO_CORR_GAP (non-zero); columns in that order
 *   rates_out    DEVICE double [n_drops][n_snr][popcount(schemes)] bit/s/Hz (NaN when not PD)
 *   status_out   DEVICE int32 [n_drops] or NULL: OR of XLMIMO_ST_* over the SNR points
 * Batches with K up to XLMIMO_MAX_USERS run one wave per drop with the matrix
 * in LDS (or registers for K <= 16).  A batch with a larger K (up to
 * XLMIMO_MAX_USERS_EXACT) runs one 512-thread workgroup per drop with the
 * matrix in a context workspace of the Gram's size (schemes XLMIMO_MZF and
 * XLMIMO_MZF_MISM are rejected there with XLMIMO_EINVAL). */
int xlmimo_zf_mmse_sumrate(xlmimo_ctx* ctx, const xlmimo_batch* batch,
                           const double* gram_true, const double* gram_filter,
                           int32_t n_snr, const double* rho, int32_t schemes,
                           double* rates_out, int32_t* status_out, void* stream);

/* Capacity-vs-N sweep of a ULA (Sec. IV-C): for every N in N_list the same
 * drops are re-evaluated with the chosen Gram form, rates are averaged over
 * drops (ergodic mean over drops whose rate is finite), and the saturation
 * point is located two ways:
 *   analytic  eqs. (15)-(16) per drop with threshold t_sat, averaged:
 *             sat_out[0] = E[y_up], sat_out[1] = E[y_down],
 *             sat_out[2] = (E[y_up] - E[y_down]) / spacing  (antennas);
 *   empirical sat_out[3 + s * n_sch + c] = first N, log-interpolated, with
 *             ergodic(N) / ergodic(N_max) >= 1 - eps_sat, for SNR s, scheme c.
 * In a closed-form sweep the schemes evaluate the closed-form Gram, except
 * when XLMIMO_MZF_MISM is asked for: then the exact FP64 Gram is computed as
 * the true channel and ZF, MMSE, MRC, CAP and the mismatched modified ZF use
 * it, while XLMIMO_MZF (nominal) keeps the closed form (one pass yields the
 * paper's comparison of Sec. V-C).
 *   form         XLMIMO_FORM_*; XLMIMO_FORM_CF_GATED_MLP (closed form XLMIMO_CF_GATED_QUAD +
 *                learned residual) needs mlp and log_var_max
 *                (see xlmimo_gram_closedform_mlp), otherwise mlp may be NULL
 *   N_list       HOST int64 [n_N], strictly ascending, each >= 1
 *   rho          DEVICE double [n_snr][total_users]
 *   ergodic_out  DEVICE double [n_N][n_snr][n_sch]
 *   sat_out      DEVICE double [3 + n_snr * n_sch]
 *   status_out   DEVICE int32 [n_N][n_drops] or NULL
 * The batch's n_elems is ignored.  Exact forms take K up to
 * XLMIMO_MAX_USERS_EXACT, closed forms up to XLMIMO_MAX_USERS. */
int xlmimo_capacity_sweep(xlmimo_ctx* ctx, const xlmimo_array* arr, int32_t n_N, const int64_t* N_list,
                          const xlmimo_batch* batch, int32_t form, xlmimo_mlp* mlp, double log_var_max,
                          int32_t n_snr, const double* rho, int32_t schemes, double t_sat, double eps_sat,
                          double* ergodic_out, double* sat_out, int32_t* status_out, void* stream);

/* ---- Learned residual correction of the closed form (not in the paper) ----
 * Per user pair i < j of a ULA drop the network sees
 *   (r_i/50, theta_i/(pi/3), r_j/50, theta_j/(pi/3), log4 N - 6, d/lambda - 1/2)
 * (r, theta: polar coordinates of the user about the array centre, theta from
 * broadside, with x the distance from the array line) and predicts
 *   delta_rho = sum_m c_m b_m,  c_m = c0_m + (network output m),  c0 = (1, 1, 0),
 * over three basis phasors b_m: the discrete sum's end-element terms at the two
 * array ends and e^{j phi(y*)} at the stationary point y*, with
 * phi(y) = (2 pi / lambda)(r_i(y) - r_j(y)) (phases computed in FP64), plus
 * s = log sigma^2.  An all-zero output is thus the analytic end correction,
 * and the network learns the deviation from it.  Network: XLMIMO_MLP_IN -> [Linear(width) +
 * GELU] x depth -> Linear(XLMIMO_MLP_OUT); BF16 weights and activations on the
 * matrix cores, FP32 accumulation; FP32 master weights and Adam state.
 * Parameters, flat FP32: per layer W (out x in, row-major) then b (out). */
/* An MLP belongs to its context: destroy it before the context. */
int     xlmimo_mlp_create(xlmimo_ctx* ctx, int32_t width, int32_t depth, xlmimo_mlp** out);
int     xlmimo_mlp_destroy(xlmimo_mlp* mlp);
int64_t xlmimo_mlp_param_count(const xlmimo_mlp* mlp);
/* HOST float [param_count]; set also resets the Adam state.  Both synchronise the device. */
int     xlmimo_mlp_set_params(xlmimo_mlp* mlp, const float* host_params);
int     xlmimo_mlp_get_params(xlmimo_mlp* mlp, float* host_params);
/* Fallback gate by antenna count.  A drop of N antennas falls back to the exact
 * Gram when any of its pairs has a predicted log-variance above
 * min(log_var_max of the call, log_var_max[b]), b the first bin with
 * N <= n_upper[b]; N above the last bound uses the call's value alone.  A
 * threshold of -inf sends every drop of its bin to the exact Gram (a batch that
 * falls back whole skips the network).  The thresholds are meant to be
 * calibrated on held-out drops with the exact Gram as the judge.
 *   n_bins       0 .. 16 (0 clears the table)
 *   n_upper      HOST int64 [n_bins], strictly ascending, >= 1
 *   log_var_max  HOST double [n_bins], not NaN (-inf allowed)
 * Takes effect for calls enqueued afterwards (a captured graph keeps the
 * table it was captured with). */
int     xlmimo_mlp_set_gate(xlmimo_mlp* mlp, int32_t n_bins, const int64_t* n_upper, const double* log_var_max);
/* Number of pairs i < j over the batch (host arithmetic, -1 on bad input). */
int64_t xlmimo_pair_count(const xlmimo_batch* batch);

/* Pair inputs of every drop, pairs drop-major and (i, j) row-major:
 *   gram_cf     DEVICE closed-form Gram (layout above)
 *   gram_exact  DEVICE exact Gram, or NULL when no targets are wanted
 *   features    DEVICE bf16 [n_pairs][XLMIMO_PAIR_FEAT_PITCH]
 *   aux         DEVICE float [n_pairs][XLMIMO_PAIR_AUX_PITCH]
 *   target      DEVICE float [n_pairs][2] = rho_exact - rho~ (complex), or NULL
 *   pair_map    DEVICE int32 [n_pairs][2] = (drop, 64 i + j) */
int xlmimo_mlp_pair_inputs(xlmimo_ctx* ctx, const xlmimo_array* arr, const xlmimo_batch* batch,
                           const double* gram_cf, const double* gram_exact, void* features, float* aux,
                           float* target, int32_t* pair_map, void* stream);

/* Mean Gaussian negative log-likelihood over n pairs and its gradient (DEVICE
 * float [param_count], or NULL to keep it internal); loss_out DEVICE double. */
int xlmimo_mlp_loss_grad(xlmimo_ctx* ctx, xlmimo_mlp* mlp, int64_t n, const void* features, const float* aux,
                         const float* target, float* grad_out, double* loss_out, void* stream);
/* One Adam step (b1 = 0.9, b2 = 0.999, eps = 1e-8) on the loss above. */
int xlmimo_mlp_train_step(xlmimo_ctx* ctx, xlmimo_mlp* mlp, int64_t n, const void* features, const float* aux,
                          const float* target, float lr, double* loss_out, void* stream);
/* n_steps Adam steps as xlmimo_mlp_train_step, enqueued in one call: step i
 * trains on the pairs [(i mod (n / batch)) batch, + batch) of the pair arrays,
 * with learning rate lr[i].
 *   lr        HOST float [n_steps], finite, >= 0
 *   loss_out  DEVICE double [n_steps] (each step's loss) or NULL */
int xlmimo_mlp_train(xlmimo_ctx* ctx, xlmimo_mlp* mlp, int64_t n, const void* features, const float* aux,
                     const float* target, int64_t batch, int64_t n_steps, const float* lr, double* loss_out,
                     void* stream);
/* Network outputs, DEVICE float [n][XLMIMO_MLP_OUT].  Widths 64, 128 and 256 run
 * one fused kernel (128 pairs per workgroup at width 256, 64 otherwise;
 * activations kept in LDS). */
int xlmimo_mlp_forward(xlmimo_ctx* ctx, xlmimo_mlp* mlp, int64_t n, const void* features, float* out,
                       void* stream);

/* Closed form (variant as in xlmimo_gram_closedform) + learned residual:
 * G_ij = G~_ij + delta_rho sqrt(G~_ii G~_jj) for every pair.  A drop with any
 * pair whose predicted log-variance exceeds log_var_max (or the threshold of its
 * N set by xlmimo_mlp_set_gate, whichever is lower) is recomputed with the
 * exact FP32H Gram and gets XLMIMO_ST_FELL_BACK in status_out (ULA only). */
int xlmimo_gram_closedform_mlp(xlmimo_ctx* ctx, const xlmimo_array* arr, const xlmimo_batch* batch,
                               int32_t variant, xlmimo_mlp* mlp, double log_var_max, double* gram_out,
                               int32_t* status_out, void* stream);

/* ---- Batching: graph capture and autotuned launch shapes (not part of the method) ----
 *
 * Graph capture records every call made on `stream` between xlmimo_graph_begin
 * and xlmimo_graph_end into one executable hipGraph that replays the whole
 * sequence with a single launch (for example a capacity sweep over
 * thousands of drops: its persistent Gram launches, rates and reductions).
 *   - `stream` must be a created (non-default) stream; while the capture is
 *     open, calls of this context on any other stream fail with XLMIMO_EINVAL.
 *   - Captured calls must be warm: run the same calls once before capturing
 *     them, so that their launch plans exist and the workspace is large enough.
 *     A call that would need a new plan, a larger workspace or a new N list,
 *     and the synchronising calls (xlmimo_mlp_create, xlmimo_mlp_set_params,
 *     xlmimo_mlp_get_params, xlmimo_mlp_train_step, xlmimo_mlp_train, xlmimo_timing_read,
 *     xlmimo_autotune_exact), fail with XLMIMO_EINVAL; xlmimo_graph_end then
 *     fails as well and no graph is made.
 *   - A graph reads and writes the same device buffers at every launch (the
 *     caller's inputs and outputs, the context's workspace): keep the
 *     caller's buffers alive and in place while the graph is used.  Replays
 *     share the context's workspace with its other calls; they are ordered on
 *     their stream like any other call.
 *   - While any graph of a context exists, workspace the context would free
 *     is kept until the context is destroyed; xlmimo_mlp_destroy and
 *     xlmimo_ctx_destroy fail with XLMIMO_EINVAL until its graphs are
 *     destroyed.
 *   - The exact-Gram kernel timing (xlmimo_timing_enable) is not recorded
 *     inside a graph. */
typedef struct xlmimo_graph xlmimo_graph;
int     xlmimo_graph_begin(xlmimo_ctx* ctx, void* stream);
int     xlmimo_graph_end(xlmimo_ctx* ctx, void* stream, xlmimo_graph** out);
int     xlmimo_graph_launch(xlmimo_graph* graph, void* stream);
int64_t xlmimo_graph_node_count(const xlmimo_graph* graph);   /* -1 for NULL */
int     xlmimo_graph_destroy(xlmimo_graph* graph);           /* waits for the device */

/* Autotune the exact-Gram launch of one batch shape.  Candidate work-item
 * lengths (1024 ... 131072 elements, powers of two) and persistent grid sizes
 * (all resident workgroups, 3/4 and 1/2 of them) are timed on `stream` (median
 * of three launches after one warm-up; the call synchronises the stream).  The
 * fastest shape is kept in the context and used by every later exact-Gram
 * launch of that shape and precision (xlmimo_gram_exact, the sweep's per-N
 * launches, the learned form's fallback).
 *   n_elems    0: the batch's own N; > 0: every drop with N = n_elems (a ULA
 *              sweep point, as xlmimo_capacity_sweep launches it)
 *   chunk_out  HOST, optional: chosen work-item length in elements
 *   grid_out   HOST, optional: chosen number of workgroups
 *   ms_out     HOST, optional: median launch time of the chosen shape
 * Results depend on the shape only through FP32/FP64 summation order (the
 * work-item partition); they stay deterministic for a given shape. */
int xlmimo_autotune_exact(xlmimo_ctx* ctx, const xlmimo_array* arr, const xlmimo_batch* batch, int64_t n_elems,
                          int32_t precision, int64_t* chunk_out, int32_t* grid_out, double* ms_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* XLMIMO_H */
