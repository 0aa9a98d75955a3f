/*
 * tsne_mi355x.h -- C ABI of the MI355X (gfx950) exact t-SNE hot path.
 *
 * The single-cell workflow profiled in the paper spends one of its most
 * GPU-intensive stages in t-SNE of PCA scores (abstract; Table 1, row 7,
 * "Umap + t-sne").  The paper names the stage but defines none of its steps,
 * so each entry point below computes the standard published definition it
 * cites:
 *   [vdMH08] van der Maaten & Hinton, JMLR 9 (2008), "Visualizing Data
 *            using t-SNE": eq. 1 (conditional P), eq. 3 (perplexity),
 *            Sec. 3.1 (symmetric P), eq. 4 (Student-t Q), eq. 5 (gradient),
 *            Sec. 3.4 / Algorithm 1 (momentum, early exaggeration).
 *   [vdM14]  van der Maaten, JMLR 15 (2014), "Accelerating t-SNE using
 *            Tree-Based Algorithms", Sec. 4.1 (sparse P on the exact
 *            k = 3*perplexity nearest-neighbour graph).
 *   [Jac88]  Jacobs, Neural Networks 1 (1988): per-parameter gains.
 *   [HMT11]  Halko, Martinsson & Tropp, SIAM Review 53 (2011), "Finding
 *            structure with randomness": Algorithm 4.4 (randomized
 *            subspace iteration), Algorithm 5.1 (direct SVD) -- tsne_pca.
 *   [LRHSK19] Linderman, Rachh, Hoskins, Steinerberger & Kluger, Nat.
 *            Methods 16 (2019), "Fast interpolation-based t-SNE for
 *            improved visualization of single-cell RNA-seq data":
 *            repulsive sums by polynomial interpolation on equispaced
 *            nodes and FFT convolution (the approximate form below).
 *   [MHM18]  McInnes, Healy & Melville, "UMAP: Uniform Manifold
 *            Approximation and Projection for Dimension Reduction",
 *            arXiv:1802.03426 (2018): local fuzzy simplicial sets and their
 *            fuzzy union (Sec. 3.1), the fitted low-dimensional similarity
 *            and the layout by SGD with negative sampling (Sec. 3.2) --
 *            the tsne_umap_* entry points.
 *   [SLF14]  Steele, Lea & Flood, "Fast splittable pseudorandom number
 *            generators", OOPSLA 2014: SplitMix64, the counter-based
 *            generator of UMAP's negative samples.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.   Every array argument is a DEVICE pointer on the current HIP
 *           device, owned by the caller, 16-byte aligned, in the layout
 *           stated.  The library never allocates or frees memory and keeps
 *           no state between calls.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default
 *           stream).  Work is enqueued and the call returns without a host
 *           synchronisation.  Scalars the host may want (nnz, Z, KL, counts)
 *           are written to caller-provided device scalars.
 * Workspace. Entry points that need scratch take (void* workspace,
 *           size_t* workspace_bytes).  With workspace == NULL the call only
 *           stores the required byte count in *workspace_bytes and returns
 *           TSNE_OK without touching the device.  Otherwise *workspace_bytes
 *           must be at least that size (else TSNE_ERR_WORKSPACE); the
 *           workspace must be device memory aligned to 256 bytes; its
 *           contents on entry are ignored.
 * Errors.   Arguments are validated before any HIP call; invalid ones
 *           return TSNE_ERR_INVALID_ARG or TSNE_ERR_UNSUPPORTED and enqueue
 *           nothing.  Then, before its first launch, a call that does device
 *           work checks the current HIP device: anything but a gfx950 (or
 *           no HIP device at all) returns TSNE_ERR_UNSUPPORTED with nothing
 *           enqueued; the answer is cached per device ordinal.  A failed
 *           launch returns TSNE_ERR_HIP and its hipError_t is kept per
 *           thread (tsne_last_hip_error).  Asynchronous device faults
 *           surface at the caller's next synchronisation.  No C++ exception
 *           crosses the ABI.
 * Non-finite inputs.  tsne_knn, tsne_kl_grad, tsne_kl_grad_fft and
 *           tsne_optimize take a nullable `nonfinite` device int64 scalar:
 *           the call zeroes it (a fill kernel on `stream`) and its kernels
 *           add the number of NaN or infinite coordinates they meet, as
 *           stated per entry point.  The computation itself goes on
 *           (non-finite values propagate); once the caller has synchronised,
 *           a nonzero count is the condition TSNE_ERR_NONFINITE names.
 * Threads.  Re-entrant; concurrent calls on different streams with
 *           disjoint buffers are safe.
 * Results.  Deterministic for fixed inputs and device: no floating-point
 *           atomics, every reduction in a fixed order.
 */
#ifndef TSNE_MI355X_H
#define TSNE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSNE_ABI_VERSION 3

#define TSNE_OK 0
#define TSNE_ERR_INVALID_ARG 1
#define TSNE_ERR_UNSUPPORTED 2
#define TSNE_ERR_WORKSPACE 3
#define TSNE_ERR_HIP 4
/* Not returned by a call (the count is on the device when it returns): the
 * status a caller reports after reading a nonzero `nonfinite` count. */
#define TSNE_ERR_NONFINITE 5
/* tsne_kl_grad_noalloc: the problem needs more than its static scratch. */
#define TSNE_ERR_SCRATCH 6

/* precision argument of tsne_knn */
#define TSNE_KNN_FP32 0 /* exact: FP32 direct differences on the VALU */
#define TSNE_KNN_BF16 1 /* BF16 MFMA candidates, FP32 exact re-rank */

/* dtype argument of the differentiation form */
#define TSNE_F32 0
#define TSNE_F64 1

/* Largest supported neighbour count k and BF16 candidate count. */
#define TSNE_MAX_K 256
/* Largest supported input dimension D. */
#define TSNE_MAX_D 256
/* BF16 path: D plus 6 norm slots must fit the 64-wide MFMA K extent. */
#define TSNE_MAX_D_BF16 58

int tsne_abi_version(void);
const char* tsne_status_string(int status);
/* hipError_t (as int) of the last TSNE_ERR_HIP returned on this thread. */
int tsne_last_hip_error(void);

/*
 * tsne_knn -- exact k nearest neighbours [vdM14 Sec. 4.1].
 * For every row i of X: the k indices j != i with the smallest squared
 * Euclidean distance d_ij = sum_c (x_ic - x_jc)^2 (the distance inside the
 * Gaussian kernel of [vdMH08] eq. 1), ordered ascending by the key
 * (d_ij, j); self is excluded by index, ties go to the smaller index.
 *
 *   X        [n][d] float, row-major, read-only.
 *   n, d     2 <= n < 2^31; 1 <= d <= TSNE_MAX_D (TSNE_MAX_D_BF16 for BF16).
 *   k        1 <= k < n, k <= TSNE_MAX_K.
 *   precision TSNE_KNN_FP32: distances are FP32 direct differences summed
 *            in dimension order; the key order is exact in that arithmetic.
 *            TSNE_KNN_BF16: X is rounded to bfloat16 (round-to-nearest-even);
 *            MFMA tiles with FP32 accumulation give the distances between
 *            rounded points; the n_cand smallest of those per row are then
 *            re-ranked by FP32 direct differences on the unrounded X and the
 *            best k kept.  An approximation: a true neighbour is lost only if
 *            bf16 rounding pushes it past rank n_cand.
 *   n_cand   BF16 only: k <= n_cand < n, n_cand <= TSNE_MAX_K (ignored for FP32).
 *   nbr_idx  [n][k] int32 out; nbr_d2 [n][k] float out (FP32 distances).
 *   nonfinite device int64 scalar out (nullable): the number of NaN or
 *            infinite entries of X (one extra read of X).  With any, the
 *            neighbour lists of the rows involved are unspecified.
 *   Invalid: NULL pointers, sizes out of range, unknown precision.
 */
int tsne_knn(const float* X, int64_t n, int32_t d, int32_t k, int32_t precision, int32_t n_cand,
             int32_t* nbr_idx, float* nbr_d2, int64_t* nonfinite, void* workspace, size_t* workspace_bytes,
             void* stream);

/*
 * tsne_calibrate_P -- perplexity calibration [vdMH08 eq. 1 and eq. 3].
 * Per row i, over its k neighbour distances (FP32 arithmetic throughout):
 * s_j = d_ij - min_l d_il, p_{j|i} = exp(-beta_i s_j) / sum_l exp(-beta_i s_l),
 * with beta_i found by bisection (start 1, bracket (0, inf), doubling until
 * bracketed) so that the entropy H = ln sum_l e^{-beta s_l} + beta sum_j p_j s_j
 * equals ln(perplexity) nats to within tol.  H is evaluated in FP32 and the
 * search stops once that evaluation is within tol - min(TSNE_CALIB_H_MARGIN,
 * tol / 2): the margin covers the FP32 evaluation error of H (sums of k
 * exponentials; a few 1e-7 at k = 90 against an FP64 evaluation), so the
 * entropy at the returned beta, evaluated in FP64 from the same FP32
 * distances, is within tol.
 * Rows that do not reach it in max_iter evaluations keep the last beta and
 * get converged = 0.  A row whose smallest distance is shared by more than
 * `perplexity` neighbours (e.g. all k distances equal) has H > ln(perplexity)
 * for every beta: its expansion stops at beta = 2^126, where P_cond is the
 * limit, uniform over those tied neighbours (0 elsewhere unless a gap
 * s_j is below about 1e-36).
 *
 *   nbr_d2     [n][k] float, read-only (any order within a row).
 *   perplexity 0 < perplexity < k.   tol > 0.   max_iter >= 1.
 *   P_cond     [n][k] float out, aligned with nbr_d2; rows sum to 1.
 *   beta       [n] float out (nullable).  converged [n] uint8 out (nullable).
 *   n_unconverged  device int32 scalar out (nullable): rows with converged 0.
 */
#define TSNE_CALIB_H_MARGIN 2e-6f

int tsne_calibrate_P(const float* nbr_d2, int64_t n, int32_t k, float perplexity, float tol, int32_t max_iter,
                     float* P_cond, float* beta, uint8_t* converged, int32_t* n_unconverged, void* stream);

/*
 * tsne_symmetrize -- symmetric joint probabilities [vdMH08 Sec. 3.1] on the
 * kNN pattern [vdM14 Sec. 4.1]: with C_ij = p_{j|i} for j in N(i) (else 0),
 * P = (C + C^T) / (2n).  Output is CSR over the union pattern with columns
 * ascending and no diagonal; val[(i,j)] == val[(j,i)] bitwise.
 *
 *   nbr_idx  [n][k] int32, read-only: k distinct indices != i per row.
 *   P_cond   [n][k] float, read-only, aligned with nbr_idx.
 *   row_ptr  [n+1] int64 out.
 *   col, val [2 n k] capacity, int32 / float out; the first nnz are used.
 *   tpos     [2 n k] capacity int32 out (nullable): tpos[e] = position of
 *            (j, i) for entry e = (i, j).
 *   nnz      device int64 scalar out: the entry count, or -1 when a
 *            neighbour list holds an index out of range, self or a repeat
 *            (the outputs are then unspecified).
 */
int tsne_symmetrize(const int32_t* nbr_idx, const float* P_cond, int64_t n, int32_t k, int64_t* row_ptr,
                    int32_t* col, float* val, int32_t* tpos, int64_t* nnz, void* workspace, size_t* workspace_bytes,
                    void* stream);

/*
 * tsne_kl_grad -- the exact t-SNE gradient [vdMH08 eq. 4 and eq. 5] with
 * early exaggeration alpha [vdMH08 Sec. 3.4], all pairs evaluated:
 *   w_ij = 1 / (1 + ||y_i - y_j||^2),  Z = sum over ordered i != j of w_ij,
 *   g_i  = 4 sum_{j != i} (alpha p_ij - w_ij / Z) w_ij (y_i - y_j)
 *        = 4 alpha sum_{e in row i} p_e w_e (y_i - y_j) - (4/Z) sum_{j != i} w_ij^2 (y_i - y_j).
 * P must be symmetric (as tsne_symmetrize produces); Q is never stored.
 * Pair terms are FP32; per-thread partial sums are folded into FP64 per
 * tile and reduced in a fixed order.
 *
 *   Y        [n][2] float (interleaved x, y), read-only.   n >= 2.
 *   row_ptr [n+1] int64, col [nnz] int32, val [nnz] float: P as CSR.
 *   exaggeration alpha (> 0); applies to the attractive term only.
 *   grad     [n][2] float out.
 *   Z        device double scalar out (nullable).
 *   kl       device double scalar out (nullable): KL(P||Q) =
 *            sum_e p_e ln p_e - sum_e p_e ln w_e + (sum_e p_e) ln Z, always
 *            with the un-exaggerated P (0 ln 0 = 0).
 *   Zrow     [n] double out (nullable): per-row sums Z_i = sum_{j != i} w_ij.
 *   nonfinite device int64 scalar out (nullable): the number of NaN or
 *            infinite coordinates of Y.
 */
int tsne_kl_grad(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                 float exaggeration, float* grad, double* Z, double* kl, double* Zrow, int64_t* nonfinite,
                 void* workspace, size_t* workspace_bytes, void* stream);

/*
 * tsne_kl_grad_noalloc -- tsne_kl_grad for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels, the same results bit
 * for bit, but the scratch is a static device array of
 * TSNE_NOALLOC_SCRATCH_BYTES held by the library on every device it runs on
 * until the process ends, instead of a caller workspace.  The call allocates
 * and frees nothing.  The caller still passes the inputs and outputs.
 *   Arguments as tsne_kl_grad, without workspace.
 *   Limit: the scratch must hold the repulsion partials (8 B per point and
 *   superblock of the all-pairs pass), plus 4 B per point and superblock
 *   when Zrow is requested; it does whenever tsne_kl_grad's own workspace
 *   query answers at most TSNE_NOALLOC_SCRATCH_BYTES, and in all for
 *   n <= 92,160 (Zrow NULL) or n <= 53,248 (Zrow given).  Larger problems
 *   return TSNE_ERR_SCRATCH before any HIP call.
 *   The first call on a device looks up the scratch's device address there
 *   (hipGetSymbolAddress, with that device current) and keeps it.
 *   Every call on one device shares that device's scratch: calls that
 *   overlap in time on one device (different streams or threads) race and
 *   give undefined results.  Nothing in the scratch needs to start at zero.
 */
#define TSNE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

int tsne_kl_grad_noalloc(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                         float exaggeration, float* grad, double* Z, double* kl, double* Zrow, int64_t* nonfinite,
                         void* stream);

/*
 * tsne_kl_grad_fft -- the t-SNE gradient of tsne_kl_grad with the repulsive
 * sums and Z approximated by FFT-accelerated polynomial interpolation
 * [LRHSK19]; the attraction (and the KL's P terms) stay exact over the CSR
 * rows.  The points' square bounding domain [lo, lo + B h]^2 (lo, hi = the
 * smallest and largest coordinate) is cut into B x B boxes of side h with
 *   B = clamp(ceil((hi - lo) / max_box_width), min_boxes, max_fft / (2 p)),
 *   h = (hi - lo) / B,
 * each box holding p x p nodes at local positions (k + 1/2) / p.  Every
 * point spreads the charges 1 and y - c (c = the domain centre) to its
 * box's nodes with tensor Lagrange weights; the node potentials of the
 * kernels 1 / (1 + r^2) and its square are circular convolutions of the
 * zero-padded node grids, done as 2-D FFTs in FP64 of size F = the smallest
 * power of two >= max(64, 2 p B) (the kernels are even, so two real grids
 * share each complex transform); each point interpolates them back:
 *   R_i = (y_i - c) phi2_i - phi3_i,  Z = sum_i phi1_i - n,
 *   g_i = 4 (alpha A_i - R_i / Z).
 * The error falls as h^p (third order for p = 3); box side 1 (the default
 * of [LRHSK19]) gives about 1e-3 relative error in R and 1e-5 in Z on
 * embeddings of a few thousand points.  Node sums are 64-bit fixed point,
 * so the result is bitwise reproducible.  The grid is set up on the device
 * from Y: the call does not synchronise.
 *
 *   Y, row_ptr, col, val, exaggeration, grad, Z, kl, nonfinite: as tsne_kl_grad.
 *   n_interp       p, nodes per box and axis, 2..5 (3).
 *   min_boxes      lower bound of B (>= 1; 50).
 *   max_box_width  upper bound of h while B < max_fft / (2 p) (> 0; 1.0).
 *   max_fft        largest F, a power of two in [64, 4096] with
 *                  2 p min_boxes <= max_fft (2048); the workspace grows as
 *                  48 max_fft^2 bytes plus 6 max_fft^2 for the node sums.
 */
int tsne_kl_grad_fft(const float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                     float exaggeration, int32_t n_interp, int32_t min_boxes, float max_box_width, int32_t max_fft,
                     float* grad, double* Z, double* kl, int64_t* nonfinite, void* workspace,
                     size_t* workspace_bytes, void* stream);

/*
 * tsne_pca -- principal components of X (the step that produces the PCA
 * scores t-SNE embeds): randomized truncated SVD of the column-centred
 * Xc = X - 1 mu^T [HMT11 Alg. 4.4 + 5.1] with a subspace of l = 64 columns:
 *   Q = orth(Xc Omega); q times: Q = orth(Xc orth(Xc^T Q));
 *   Z = Xc^T Q, Z^T Z = U diag(s^2) U^T (s descending);
 *   components = (Z U diag(1/s))^T, scores = Q U diag(s) (= Xc components^T
 *   when Q spans the range of Xc).
 * orth() is the Q factor with a positive R diagonal (CholeskyQR2 here).
 * Sign convention: each component's entry of largest magnitude is positive
 * (the first on ties); the scores follow.  Products with X run on the FP32
 * matrix cores, the 64 x 64 steps in FP64; bitwise reproducible.  Xc must
 * have rank >= 64 (else the trailing directions are not defined).
 *
 *   X          [n][g] float, read-only; 64 <= n <= 65535 * 2048, 64 <= g <= 2^20.
 *   k          components returned, 1..64.
 *   q          power iterations, 0..16 (2).
 *   omega      [g][64] float, read-only: the random test matrix (the caller
 *              draws it, e.g. i.i.d. N(0, 1)).
 *   scores     [n][k] float out.
 *   components [k][g] float out (orthonormal rows).
 *   singular_values [k] double out (device).
 *   mean       [g] float out: the column means.
 */
int tsne_pca(const float* X, int64_t n, int32_t g, int32_t k, int32_t q, const float* omega, float* scores,
             float* components, double* singular_values, float* mean, void* workspace, size_t* workspace_bytes,
             void* stream);

/*
 * tsne_step -- one optimiser step, gradient descent with momentum
 * [vdMH08 Algorithm 1] and adaptive gains [Jac88], elementwise over the 2n
 * coordinates, in place, FP32:
 *   gain  <- (grad * update < 0) ? gain + gain_inc : gain * gain_dec
 *   gain  <- max(gain, min_gain)
 *   update <- momentum * update - lr * gain * grad
 *   Y     <- Y + update
 *   Y, update, gains, grad  [n][2] float (grad read-only).
 */
int tsne_step(float* Y, float* update, float* gains, const float* grad, int64_t n, float lr, float momentum,
              float gain_inc, float gain_dec, float min_gain, void* stream);

/* Optimiser schedule of tsne_optimize [vdMH08 Sec. 3.4, Algorithm 1; Jac88]. */
typedef struct tsne_schedule {
  float lr;                   /* learning rate (200) */
  float exaggeration;         /* alpha while t < exaggeration_iters (12) */
  int32_t exaggeration_iters; /* (100) */
  float momentum_early;       /* momentum while t < exaggeration_iters (0.5) */
  float momentum_late;        /* momentum afterwards (0.8) */
  float gain_inc;             /* (0.2) */
  float gain_dec;             /* (0.8) */
  float min_gain;             /* (0.01) */
} tsne_schedule;

/*
 * tsne_optimize -- iterations t = t_begin .. t_end - 1 of the optimiser
 * [vdMH08 Algorithm 1], enqueued from native code: per iteration the
 * gradient of tsne_kl_grad with alpha_t = (t < exaggeration_iters ?
 * exaggeration : 1), then the update of tsne_step with momentum_t =
 * (t < exaggeration_iters ? momentum_early : momentum_late).  The step runs
 * inside the gradient's last pass, and Y alternates with a workspace copy
 * (copied back at the end when the count is odd).  The attraction term is
 * summed inside the all-pairs pass from a copy of P's upper triangle grouped
 * by superblock pair (built once per call), in 64-bit fixed point
 * (resolution 2^-56) and then rounded once, so it can differ from
 * tsne_kl_grad's FP32 sum by FP32 rounding.  Logging the KL adds a CSR
 * pass at the same Y and leaves the trajectory unchanged.  Deterministic.
 *   Y, update, gains  [n][2] float, updated in place (Y holds the result
 *                     when the enqueued work completes).  P as for
 *                     tsne_kl_grad, with a symmetric pattern, values >= 0
 *                     and every row summing to at most 1 (true for the
 *                     output of tsne_symmetrize).
 *   nnz       stored entries of P (row_ptr[n]); it sizes the workspace.
 *             The call cannot read row_ptr[n] without synchronising, so it
 *             trusts nnz: a larger value only enlarges the workspace; a
 *             smaller one leaves the job-grouped copy of P too short, and
 *             the entries past its end are dropped from the attraction
 *             (no fault, but not the gradient stated above).
 *   schedule  host pointer, read before the call returns.
 *   kl_log    device double array of (t_end - t_begin) entries (nullable):
 *             with log_every > 0, entry t - t_begin receives KL(P||Q) for the
 *             iterations with (t + 1) % log_every == 0; others are untouched.
 *   events    host array of 2 (t_end - t_begin) hipEvent_t handles (nullable;
 *             NULL entries skipped): events[2 (t - t_begin)] and [.. + 1] are
 *             recorded on `stream` right before and right after iteration
 *             t's all-pairs repulsion kernel (the dominant cost), for timing.
 *   nonfinite device int64 scalar out (nullable): the number of NaN or
 *             infinite coordinates among the positions the iterations
 *             produce, summed over the iterations (a non-finite input Y
 *             makes every later position non-finite, so it is counted too).
 */
int tsne_optimize(float* Y, float* update, float* gains, int64_t n, const int64_t* row_ptr, const int32_t* col,
                  const float* val, int64_t nnz, int32_t t_begin, int32_t t_end, const tsne_schedule* schedule,
                  int32_t log_every, double* kl_log, void* const* events, int64_t* nonfinite, void* workspace,
                  size_t* workspace_bytes, void* stream);

/*
 * Differentiation form.  KL(P||Q) as a function of the embedding Y and of
 * the stored values p_e of a CSR P whose pattern is symmetric (tpos valid);
 * the values need be neither symmetric nor normalised:
 *   C = sum_e p_e ln p_e - sum_e p_e ln w_e + S ln Z,   S = sum_e p_e,
 * the KL of [vdMH08] eq. 2 written for stored entries.  Exact derivatives:
 *   dC/dy_i = 2 sum_{e=(i,b)} p_e w_e (y_i - y_b) + 2 sum_{e=(a,i)} p_e w_e (y_i - y_a)
 *             - (4 S / Z) sum_{j != i} w_ij^2 (y_i - y_j),
 *   dC/dp_e = 1 + ln p_e - ln w_e + ln Z.
 * The all-pairs terms are recomputed tile by tile (Q is never stored).
 * dtype TSNE_F32 or TSNE_F64 selects float or double for Y, val, C, gC, dY,
 * dP (one templated kernel source).  Stored p_e must be > 0.
 *
 * tsne_kl_forward:  C device scalar out (dtype); Z device double out (nullable).
 * tsne_kl_backward: gC device scalar (dtype) in; dY [n][2] out; dP [nnz] out
 *                   (nullable), both scaled by gC.
 */
int tsne_kl_forward(int32_t dtype, const void* Y, int64_t n, const int64_t* row_ptr, const int32_t* col,
                    const void* val, void* C, double* Z, void* workspace, size_t* workspace_bytes, void* stream);
int tsne_kl_backward(int32_t dtype, const void* Y, int64_t n, const int64_t* row_ptr, const int32_t* col,
                     const void* val, const int32_t* tpos, const void* gC, void* dY, void* dP, void* workspace,
                     size_t* workspace_bytes, void* stream);

/*
 * UMAP on the kNN graph [MHM18].  The neighbour lists are those of tsne_knn
 * (self excluded, squared Euclidean distances); the embedding is 2-D.
 *
 * tsne_umap_fit_ab -- host only (no device work): a, b of the similarity
 * Phi(d) = 1 / (1 + a d^2b) fitted by least squares (Levenberg-Marquardt
 * from a = b = 1) to Psi(d) = 1 for d <= min_dist, exp(-(d - min_dist))
 * beyond, over the 300 points d = 3 m / 299 [MHM18] Sec. 3.2.
 *   min_dist  in [0, 3).  a, b host doubles out.
 *
 * tsne_umap_weights -- the local fuzzy simplicial set of every row [MHM18]
 * Sec. 3.1: with d_j = sqrt(d2_j) (FP64), rho = the smallest positive d_j
 * (0 if none), sigma the root of sum_j exp(-max(0, d_j - rho) / sigma) =
 * log2(k) (FP64 bisection; sigma >= 1e-3 mean_j d_j, or 1e-3 when every
 * d_j is 0, and sigma stays at that floor when the floor already meets the
 * target), w_j = exp(-max(0, d_j - rho) / sigma).
 *   nbr_d2    [n][k] float: squared distances of the neighbour lists.
 *   rho, sigma [n] float out; w [n][k] float out (row-aligned with nbr_d2).
 *   n >= 1, 1 <= k <= TSNE_MAX_K.  One launch, no workspace.
 *
 * tsne_umap_fuzzy_union -- B = A + A^T - A o A^T [MHM18] Sec. 3.1 on the
 * union of the kNN patterns: the arguments, outputs, workspace, limits and
 * error behaviour of tsne_symmetrize with the directed weights w in place
 * of P_cond; entry (i, j) holds (a + a') - a a' with a = w_{i->j}, a' =
 * w_{j->i} (0 when absent), the same FP32 value in rows i and j.
 *
 * tsne_umap_layout -- epochs [epoch_begin, epoch_end) of the layout
 * [MHM18] Sec. 3.2, in place on Y.  Epoch t: learning rate alpha =
 * alpha0 (1 - t / n_epochs); stored entry e = (i, j) of the graph is
 * sampled when floor((t + 1) r_e) > floor(t r_e) with r_e = val_e / max val
 * (FP32 division and products), so it is sampled floor(n_epochs r_e) times
 * in all.  A sampled entry adds alpha clip(c_a (y_i - y_j)) to y_i and
 * subtracts it from y_j, c_a = -2ab d^2(b-1) / (1 + a d^2b), then for
 * p < neg_rate the vertex c = ((z >> 32) n) >> 32 of the SplitMix64 output z
 * [SLF14] for seed and counter (t nnz + e) neg_rate + p (skipped if c = i)
 * adds alpha clip(c_r (y_i - y_c)) to y_i, c_r = 2b / ((1e-3 + d^2)(1 +
 * a d^2b)); no step at distance 0; clip to [-4, 4] per coordinate.  All
 * steps of an epoch are evaluated at the epoch's starting Y and summed in
 * 64-bit fixed point (2^-32), so an epoch is exact in its sums and bitwise
 * reproducible; epochs run in order on `stream`.
 *   Y         [n][2] float, in place.  2 <= n < 2^31.
 *   row_ptr, col, val  CSR graph ([n+1] int64, [nnz] int32, [nnz] float),
 *             values >= 0 with a positive maximum (the output of
 *             tsne_umap_fuzzy_union); nnz = row_ptr[n] >= 1.
 *   symmetric 1: the caller guarantees a symmetric pattern with equal FP32
 *             values in (i, j) and (j, i) (true of tsne_umap_fuzzy_union's
 *             output); then each vertex takes twice its own attractive
 *             steps instead of receiving the reverse entries' steps -- the
 *             same value bit for bit -- and the epoch scatters nothing.
 *             0: any graph; the steps into y_j are scattered with 64-bit
 *             integer atomics.  Both give identical results on a symmetric
 *             graph; 1 on a graph that is not symmetric gives undefined
 *             results (not those stated above).
 *   a, b > 0; alpha0 >= 0; 0 <= neg_rate <= 64; n_epochs >= 1;
 *   0 <= epoch_begin <= epoch_end <= n_epochs.  seed: the generator's seed.
 *   Workspace: 24 n bytes + 1 KiB.
 */
int tsne_umap_fit_ab(double min_dist, double* a, double* b);
int tsne_umap_weights(const float* nbr_d2, int64_t n, int32_t k, float* rho, float* sigma, float* w, void* stream);
int tsne_umap_fuzzy_union(const int32_t* nbr_idx, const float* w, int64_t n, int32_t k, int64_t* row_ptr,
                          int32_t* col, float* val, int32_t* tpos, int64_t* nnz, void* workspace,
                          size_t* workspace_bytes, void* stream);
int tsne_umap_layout(float* Y, int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val, int64_t nnz,
                     int32_t symmetric, double a, double b, double alpha0, int32_t neg_rate, int32_t n_epochs,
                     int32_t epoch_begin, int32_t epoch_end, uint64_t seed, void* workspace, size_t* workspace_bytes,
                     void* stream);

/*
 * Resource monitor of a workload (the analogue of the paper's GPU monitor,
 * Section 2, and of its CPU monitor of the workload's process, Section 3.2).
 * Host-only calls, no device work.
 *
 * tsne_monitor_start -- starts a sampler thread.  Every period_s seconds
 * (on a fixed grid from the start) it appends to samples_csv one row of
 *   t_s, gfx_pct, umc_pct, vram_used_bytes, vram_total_bytes, temp_edge_c,
 *   temp_hotspot_c, temp_vram_c, power_w, proc_cpu_pct, proc_rss_bytes,
 *   hip_used_bytes, sample_us
 * (seconds since start, taken after the row's last reading; graphics /
 * memory-controller activity, VRAM and temperatures and socket power of
 * HIP device hip_device from amd-smi;
 * CPU share over the last period and resident bytes of process pid from
 * /proc, pid 0 = the calling process; device memory in use as the HIP
 * runtime reports it, total - free; the time one sample took).  The
 * activity and power readings are the device's own running averages and
 * trail a change of load by a fraction of a second.  GPU
 * columns are nan when amd-smi, the device (hip_device < 0 for none) or a
 * sensor is unavailable.  events_csv receives (t_s, name) rows: "start" at 0,
 * the timestamps, "stop" at the end.  Both files are created (truncated)
 * and flushed row by row.
 *   period_s in [1e-3, 3600]; pid >= 0; *out receives the handle.
 *   Errors: TSNE_ERR_INVALID_ARG (bad argument, a file cannot be opened,
 *   or no thread could be started).
 * tsne_monitor_timestamp -- appends (now, name) to the events; commas,
 *   quotes and line breaks in name become '_'.  Thread-safe.
 * tsne_monitor_has_gpu -- 1 when the GPU columns are being sampled.
 * tsne_monitor_stop -- takes a last sample, writes "stop", closes the files
 *   and frees the handle; the handle must not be used afterwards (and no
 *   timestamp may race with the stop).
 * tsne_monitor_steps -- the step table: step k < n_events - 1 is the
 *   interval [events[k], events[k + 1]) (each interval assigned to the first
 *   of its two timestamps, as the paper's workflow figure does); over the
 *   samples t[i] in it, count[k], and per field q the mean and maximum of
 *   the finite values[i][q] (nan when none): mean, maxv [n_events - 1][n_fields].
 *   t ascending [n], values [n][n_fields] (host arrays), events ascending
 *   (n_events >= 2).
 */
typedef struct tsne_monitor tsne_monitor;
int tsne_monitor_start(double period_s, int32_t hip_device, int32_t pid, const char* samples_csv,
                       const char* events_csv, tsne_monitor** out);
int tsne_monitor_timestamp(tsne_monitor* monitor, const char* name);
int tsne_monitor_has_gpu(const tsne_monitor* monitor);
int tsne_monitor_stop(tsne_monitor* monitor);
int tsne_monitor_steps(const double* t, const double* values, int64_t n, int32_t n_fields, const double* events,
                       int64_t n_events, int64_t* count, double* mean, double* maxv);

#ifdef __cplusplus
}
#endif

#endif /* TSNE_MI355X_H */
