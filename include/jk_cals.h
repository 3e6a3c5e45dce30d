/*
 * jk_cals.h -- C ABI of the MI355X (gfx950) JK-CALS hot path.
 *
 * JK-CALS fits all leave-one-out jackknife submodels of a CP model at once
 * (Psarras, Karlsson, Bro, Bientinesi, "Accelerating jackknife resampling for
 * the Canonical Polyadic Decomposition", arXiv 2112.03985, Sec. 4.1, Alg. 3).
 * Every submodel keeps its own factor matrices; the factors of all models
 * are stored side by side as column blocks of one "multi-factor" per mode,
 * and each mode's MTTKRP of all models is one fused product of the mode-n
 * unfolding of the FULL tensor with the column-concatenated Khatri-Rao
 * products (Alg. 3, MTTKRP step).  A submodel that leaves out sample p of
 * the sampled mode keeps a row of zeros at index p of that mode's factor
 * (Case II), and the fused MTTKRP's row p is discarded for that model when
 * the sampled mode itself is updated (Case I).  Delete-d jackknife keeps d
 * such rows per submodel (Sec. 4.1, closing remark).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Tensor T of order N (2..4) with sizes I_1..I_N: device memory, column-major
 *   with i_1 fastest (Eq. (3)): element (i_1..i_N) at offset
 *   i_1 + I_1*(i_2 + I_2*(i_3 + ...)).  float64 or float32 (tensor_dtype).
 * Models: K models; model k has rank R_k (1..JKC_MAX_RANK) and leaves out
 *   the samples P_k of the sampled mode listed in left_out (one per model,
 *   or d per model with delete_d = d; -1: full model, keeps all).
 *   "The left-out rows of model k" below are the rows P_k of the sampled
 *   mode in model k's columns.
 *   Model k owns columns [off_k, off_k + R_k) with off_k = R_0+...+R_{k-1}.
 *   C = R_0 + ... + R_{K-1}.
 * Factors, MTTKRP results and gradients: device float64, row-major
 *   I_n x C (C contiguous, leading dimension C).
 * Modes are 0-based: mode 0 is the paper's mode 1.
 * Streams: every asynchronous call is enqueued on problem->stream (a
 *   hipStream_t; NULL means the default stream).
 * Memory: the library never allocates device memory.  The caller provides
 *   one workspace of jk_cals_workspace_size() bytes (256-byte aligned) that
 *   must outlive the context.  Inputs are copied into it at init unless
 *   copy_tensor == 0, in which case the tensor is read in place and must
 *   stay valid and unchanged for the life of the context.
 * Errors: every entry point validates all arguments before it enqueues any
 *   device work; on a non-OK status nothing has been enqueued and no state
 *   has changed, and jk_cals_last_error() describes the problem.  A HIP
 *   failure returns JKC_EDEVICE.  Numerical trouble inside a model (a
 *   singular normal matrix, a non-finite value) is not an error: it is
 *   reported per model in the status word.  Nothing is printed.
 * Threads: a context is not thread-safe; distinct contexts are independent.
 */
#ifndef JK_CALS_H
#define JK_CALS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JKC_MAX_ORDER 4
#define JKC_MAX_RANK 32

typedef struct jkc_ctx jkc_ctx;

typedef enum {
  JKC_OK = 0,
  JKC_EINVAL = -1,        /* an argument is invalid                         */
  JKC_ENOMEM = -2,        /* workspace smaller than jk_cals_workspace_size  */
  JKC_EDEVICE = -3,       /* a HIP runtime call failed                       */
  JKC_ESTATE = -4,        /* call not valid in the context's current state  */
  JKC_EUNSUPPORTED = -5   /* valid request the library does not provide      */
} jkc_status;

typedef enum {
  JKC_FP64 = 0,           /* MTTKRP in float64 MFMA, float64 accumulation    */
  JKC_SPLIT_BF16X3 = 1,   /* MTTKRP with each operand split into two
                             bfloat16 terms and three MFMA products
                             (hi*hi + hi*lo + lo*hi), float32 accumulation
                             flushed to float64; everything else float64.
                             ~2^-17 relative per product: normwise MTTKRP
                             error a few 1e-6, up to ~1e-5 when the sums
                             cancel strongly                                */
  JKC_SPLIT_BF16X6 = 2    /* three bfloat16 terms per operand, the six
                             products down to 2^-16 magnitude: ~2^-23
                             relative per product; 2x the MFMA work of
                             JKC_SPLIT_BF16X3                               */
} jkc_precision;

typedef enum { JKC_TENSOR_F64 = 0, JKC_TENSOR_F32 = 1 } jkc_tensor_dtype;

/* Per-model status bits (jk_cals_fit / jk_cals_get_status). */
#define JKC_ST_CONVERGED 1u   /* |fit_t - fit_{t-1}| < tol after sweep t >= 2 */
#define JKC_ST_FALLBACK 2u    /* an update used the eigen pseudoinverse       */
#define JKC_ST_NONFINITE 4u   /* the model's error became NaN/Inf; frozen     */

typedef struct {
  int32_t order;               /* N, 2..JKC_MAX_ORDER                         */
  const int64_t *dims;         /* host [N], each >= 1                         */
  int32_t sampled_mode;        /* n-hat, 0-based, in [0, N)                   */
  int32_t num_models;          /* K >= 1                                      */
  const int32_t *ranks;        /* host [K], 1..JKC_MAX_RANK                    */
  const int32_t *left_out;     /* host [K x d] row-major, d = max(1,
                                  delete_d): model k leaves out the samples
                                  left_out[k*d .. k*d+d-1] of the sampled
                                  mode, all distinct and in
                                  [0, dims[sampled_mode]), or all -1 (a model
                                  fitted to all of T)                        */
  int32_t tensor_dtype;        /* jkc_tensor_dtype                            */
  int32_t precision;           /* jkc_precision                               */
  int32_t copy_tensor;         /* 1: copy T into the workspace; 0: use in place
                                  (JKC_FP64 only)                             */
  void *stream;                /* hipStream_t, NULL = default stream          */
  int32_t delete_d;            /* samples left out per submodel: 0 or 1 =
                                  leave-one-out, d > 1 = delete-d jackknife
                                  (Sec. 4.1: d zero rows padded and kept zero
                                  instead of one); d < dims[sampled_mode]   */
  int32_t tree_max_gib;        /* cap on the shared contraction W of 3-way
                                  float64 sweeps (jk_cals_set_mttkrp_tree) in
                                  GiB of workspace: 0 = default (64), < 0 =
                                  never hold W (fused MTTKRP on every mode) */
} jkc_problem;

/* Bytes of device workspace the problem needs.  Host only, no device work. */
jkc_status jk_cals_workspace_size(const jkc_problem *prob, size_t *bytes);

/* Create a context (Alg. 3, initialisation of the multi-factors).
 *   tensor : device, layout above.
 *   init   : host array [N] of device pointers; init[n] is I_n x C float64,
 *            row-major.  The left-out rows of model k's block in the sampled
 *            mode are zeroed by the library (the inserted zero rows), so the
 *            caller may pass an unzeroed parent initialisation.
 *   workspace : device, >= jk_cals_workspace_size bytes, 256-byte aligned.
 *   out    : receives the context.  Owned by the caller; free with
 *            jk_cals_destroy.
 * Enqueues the tensor copy (or bfloat16 split), the slice norms
 * ||T_{-P_k}||^2 used by the submodel error (Alg. 3, error step), factor
 * packing and the initial Gram matrices.  Asynchronous on the stream. */
jkc_status jk_cals_init(const jkc_problem *prob, const void *tensor,
                        const double *const *init, void *workspace,
                        size_t ws_bytes, jkc_ctx **out);

/* The fused MTTKRP of Alg. 3 for one mode, at the context's current factors:
 * out = T_(mode) (multi-factor Khatri-Rao product), with the left-out rows
 * of model k's columns set to 0 when mode == sampled_mode (Case I).
 *   out : device, I_mode x C float64, row-major.  Asynchronous. */
jkc_status jk_cals_mttkrp(jkc_ctx *ctx, int32_t mode, double *out);

/* Run nsweeps full ALS sweeps (Alg. 3, one pass of the repeat loop each) for
 * every model that is not frozen, with no convergence test (the fixed
 * iteration protocol of Sec. 5.1).  After the last sweep, if fit != NULL,
 * fit[k] (device [K] float64) receives 1 - ||T_{-P_k} - model|| / ||T_{-P_k}||.
 * Asynchronous. */
jkc_status jk_cals_sweep(jkc_ctx *ctx, int32_t nsweeps, double *fit);

/* Iterate until every model has converged (|delta fit| < tol after at least
 * two sweeps; converged models are frozen individually) or max_iters sweeps
 * were run (Alg. 3 stopping rule; tol <= 0 disables the test).  Synchronous.
 *   iters, status : host [K] int32 (may be NULL); fit : host [K] (may be
 *   NULL).  status holds JKC_ST_* bits. */
jkc_status jk_cals_fit(jkc_ctx *ctx, int32_t max_iters, double tol,
                       int32_t *iters, double *fit, int32_t *status);

/* Copy the current factor of `mode` (device I_mode x C, row-major; columns
 * unit-norm after any sweep) and, if lambda != NULL, the column weights
 * lambda (device [C]; the model is [[lambda; U_1..U_N]]).  Asynchronous. */
jkc_status jk_cals_get_factors(jkc_ctx *ctx, int32_t mode, double *out,
                               double *lambda);

/* Replace the factor of `mode` (device I_mode x C) and, if lambda != NULL,
 * lambda (device [C]); the left-out rows of the sampled mode are re-zeroed and
 * the mode's Gram matrices are recomputed.  Asynchronous. */
jkc_status jk_cals_set_factors(jkc_ctx *ctx, int32_t mode, const double *in,
                               const double *lambda);

/* Per-model error e_k, fit_k (device [K] each, may be NULL) and status words
 * and iteration counts (device [K] int32, may be NULL).  Asynchronous. */
jkc_status jk_cals_get_status(jkc_ctx *ctx, double *err, double *fit,
                              int32_t *status, int32_t *iters);

/* Least-squares CP loss f_k = 1/2 ||T_{-P_k} - [[U^(k)]]||^2 per model for
 * the context's factors with lambda folded into the last mode (the
 * all-at-once formulation the paper cites in Sec. 2), and its gradient
 * dF/dU_n = U_n H_n - M_n for every mode (an all-mode MTTKRP: fused per
 * mode, through the shared contraction of jk_cals_set_mttkrp_tree, or in one
 * pass over T, jk_cals_set_allmode), with the left-out rows of the sampled
 * mode held at 0.  lambda is folded into the
 * last factor first (and reset to 1).  loss: device [K] (may be NULL).  The
 * gradients stay in the workspace for jk_cals_get_grad.  Asynchronous. */
jkc_status jk_cals_loss_grad(jkc_ctx *ctx, double *loss);

/* out = weights[k] * (gradient of mode `mode`) on model k's columns, from the
 * last jk_cals_loss_grad.  weights: device [K] or NULL (all ones).
 * out: device I_mode x C.  Asynchronous. */
jkc_status jk_cals_get_grad(jkc_ctx *ctx, int32_t mode, const double *weights,
                            double *out);

/* out(i, c) = weights[k] * src(i, c) for every column c of model k: the
 * chain rule of a loss that weights model k's CP loss by weights[k] (the
 * backward of the per-model loss; Sec. 2 cites gradient-based CP), applied to
 * gradients a caller copied out with jk_cals_get_grad(..., NULL, ...).
 * src, out: device rows x C row-major (src == out allowed); weights: device
 * [K] or NULL (all ones).  EINVAL for rows < 0 or NULL buffers when rows > 0.
 * Asynchronous on the context's stream. */
jkc_status jk_cals_scale_columns(jkc_ctx *ctx, int32_t rows, const double *src,
                                 const double *weights, double *out);

/* Gradient refinement: fold lambda into the last factor, fix the step
 * eta_k = 1 / sum_n ||H_n^(k)||_F from the current factors, then take
 * `steps` steps U_n <- U_n - eta_k dF/dU_n (all modes at once).  If loss is
 * not NULL it receives the loss at the final factors (device [K]).
 * Asynchronous. */
jkc_status jk_cals_refine(jkc_ctx *ctx, int32_t steps, double *loss);

/* Jackknife uncertainty of the factors (Alg. 2: the permutation and scale
 * adjustment of every fitted submodel against the overall model, then the
 * standard deviation of each factor matrix except the sampled mode's over
 * the submodels), from the context's current factors.
 *   ref:   index of the reference model (normally the one with
 *          left_out = -1, fitted to all of T);
 *   first, count: the set of submodels, models first .. first+count-1, all
 *          of the reference's rank R (their columns are contiguous);
 *   std:   host array[N] of device pointers; std[n] (n != sampled mode)
 *          receives S_n, I_n x R row-major; std[sampled mode] is not used
 *          (may be NULL);
 *   perm:  device [count x R] int32 or NULL: perm[j*R + s] is the component
 *          of model first+j matched to reference component s;
 *   sign:  device [N x count x R] or NULL: sign[(n*count + j)*R + s] = +1 or
 *          -1, the sign applied to that matched column in mode n (+1 for the
 *          sampled mode and for zero columns).
 * Matching (a reading; the paper defers to its citation): congruence of a
 * submodel component with a reference component = product over the
 * non-sampled modes of the cosines of their loading vectors; the assignment
 * maximising the sum of absolute congruences is solved exactly.  Scale
 * adjustment: non-sampled loading vectors scaled to unit norm, sign chosen
 * so the inner product with the matched reference vector is >= 0.
 * Deviation: S = sqrt((count-1)/count * sum_j (theta_j - mean)^2).
 * JKC_EINVAL for an out-of-range ref or set, a rank mismatch or a missing
 * std[n].  Asynchronous; the context's workspace holds the matching. */
jkc_status jk_cals_jackknife_std(jkc_ctx *ctx, int32_t ref, int32_t first, int32_t count,
                                 double *const *std, int32_t *perm, double *sign);

/* Convergence compaction in jk_cals_fit (on by default): at every
 * convergence check, once a fifth of the columns the fused MTTKRP covers
 * belong to converged or non-finite (frozen) models, the models still being
 * fitted are moved to the front of the multi-factors so the MTTKRP covers
 * only their columns; the canonical column layout is restored before
 * jk_cals_fit returns.  Every model's arithmetic is unchanged (its columns'
 * sums run in the same order wherever they sit), so results are bitwise the
 * same with compaction on or off.  enable: 0 or 1 (JKC_EINVAL otherwise).
 * Host only. */
jkc_status jk_cals_set_compaction(jkc_ctx *ctx, int32_t enable);

/* Time each candidate MTTKRP tiling of every mode on this problem and keep
 * the fastest (restores the factors it started with).  Synchronous.
 * Optional: a context works with its built-in choice without it. */
jkc_status jk_cals_tune(jkc_ctx *ctx, int32_t reps);

/* The current tiling of `mode` as text, e.g. "f64 wm2 wn2 tm2 tn2 bk16 s8";
 * mode = N names the shared partial contraction of 3-way sweeps ("tree ...",
 * "" when sweeps do not use it).  "" for other modes or a NULL context.  The
 * string stays valid until the next call on this context. */
const char *jk_cals_describe(jkc_ctx *ctx, int32_t mode);

/* Choose the per-model update (Alg. 3 update step): 0 = one block per
 * model with its rows staged in LDS, the split-K reduction fused in when
 * there are at most two partials (default; falls back to 1 when the rows
 * do not fit LDS); 1 = a separate reduction kernel, then one block per model
 * working in global memory; 2 = row-parallel: one kernel per (model, 64-row
 * chunk) sums the split-K partials, solves and stages the chunk's rows, a
 * second normalises them and writes lambda, the Gram block and the error
 * (more blocks, but slower on the benchmark shape).  All three compute the same
 * update; sums run in fixed orders (bitwise repeatable per choice), which
 * differ between choices only by rounding.  EINVAL for other values.
 * Host only. */
jkc_status jk_cals_set_update_kernel(jkc_ctx *ctx, int32_t which);

/* Shared partial contraction of a 3-way float64 sweep: an extension beyond
 * Alg. 3, which computes every mode's MTTKRP separately.  The MTTKRPs of
 * Alg. 1 inside the concurrent sweep are evaluated as a two-level dimension
 * tree (the reuse of partial MTTKRPs of Phan et al., the paper's reference
 * for the error identity; modes numbered from 0): at mode 0 the tensor is
 * contracted once with
 * the last factor, W(i,j,c) = sum_k T(i,j,k) U_2(k,c) for all active
 * columns, and M_0 = sum_j W U_1, M_1 = sum_i W U_0 (U_0 just updated) are
 * read from W; mode 2 keeps the fused MTTKRP.  The results equal the fused
 * path's up to rounding (different summation order).  enable = 1 is the
 * default when the problem is 3-way, float64, and W ([I_0 I_1] x ldc
 * doubles, part of the workspace) fits jkc_problem.tree_max_gib (default
 * 64 GiB) with I_0, I_1 <= 100000;
 * JKC_EUNSUPPORTED for enable = 1 otherwise, EINVAL for other values.
 * The all-mode MTTKRP of jk_cals_loss_grad / jk_cals_refine uses the same
 * W (the factors are fixed there, so it serves modes 0 and 1 and the tensor
 * is read twice instead of three times); jk_cals_mttkrp always runs the
 * fused MTTKRP.  Host only. */
jkc_status jk_cals_set_mttkrp_tree(jkc_ctx *ctx, int32_t enable);

/* All-mode MTTKRP of jk_cals_loss_grad / jk_cals_refine in one pass over the
 * tensor (the gradient of the all-at-once CP loss, Sec. 2, needs every
 * mode's MTTKRP at the same factors): a tile of T staged once feeds the
 * fused MTTKRP of mode 0 and the mode-0 contraction Z = T x_0 U_0 on the
 * float64 matrix cores, from which the other modes follow by per-column
 * products -- 4 C P matrix-core flops for all modes instead of 2 N C P.
 * Available for 3- and 4-way float64 problems with at most 256 rows in mode
 * 0, a tensor below 2^31 bytes and a block that fits in LDS; the default
 * where no shared contraction is held (4-way problems, 3-way problems whose W
 * does not fit), where it is the faster path.  enable = 0 returns to the
 * per-mode path (the shared contraction where held, else the fused MTTKRP of
 * every mode).  Results agree up to rounding (summation order).
 * JKC_EUNSUPPORTED for enable = 1 on other problems, EINVAL for other
 * values.  Host only. */
jkc_status jk_cals_set_allmode(jkc_ctx *ctx, int32_t enable);

/* Replay multi-sweep runs of jk_cals_sweep from a HIP graph of one sweep,
 * captured on first use (enable = 1), or launch every kernel directly
 * (enable = 0, the default: on MI355X the direct launches of the benchmark
 * sweep finish about 3 % sooner than the graph's).  The results are
 * identical.  Host only. */
jkc_status jk_cals_set_sweep_graph(jkc_ctx *ctx, int32_t enable);

/* Number of MTTKRP tilings compiled for the context's precision (0 if ctx is
 * NULL). */
int32_t jk_cals_num_tilings(jkc_ctx *ctx);

/* Force tiling `variant` (0 .. num_tilings-1) with `splits` K chunks
 * (clamped to 1 .. the context's limit) for `mode`; mode = N selects the
 * shared partial contraction W of 3-way float64 sweeps (splits must be 1;
 * JKC_EINVAL when the context holds no W).  Any tiling gives the
 * same result up to the order of the float64 sums.  JKC_EINVAL for a
 * buffer-load tiling (its description ends in "-buffer") when the tensor or
 * a multi-factor takes 2^31 bytes or more, and for the narrow vector-ALU
 * tiling ("valu-narrow": a streaming pass over T for problems of at most 16
 * columns, the plain per-submodel ALS of Alg. 2) when C > 16 or mode 0 has
 * more than 256 rows (128 with more than 8 columns).  Host only. */
jkc_status jk_cals_set_tiling(jkc_ctx *ctx, int32_t mode, int32_t variant, int32_t splits);

/* Kernel timing of the fused MTTKRP (the dominant kernel; Alg. 3, MTTKRP
 * step): while enabled, every MTTKRP launch of this context is bracketed by a
 * pair of HIP events on the context's stream, stamped by the dispatches
 * themselves (at most 65536 launches are kept).  A launch whose split-K
 * partials are summed by a separate reduction is timed from the start of the
 * MTTKRP to the end of that reduction; the shared contraction W of 3-way
 * sweeps is timed on its own.  Host only. */
jkc_status jk_cals_profile(jkc_ctx *ctx, int32_t enable);

/* Synchronise the stream, then report per slot the number of launches timed
 * since the last read and their summed time in milliseconds: slot n < N is
 * the fused MTTKRP of mode n (with its reduction, as above), slot N the
 * shared contraction W (launches: host [N+1] int64, ms: host [N+1] float64;
 * either may be NULL).  Resets the counts. */
jkc_status jk_cals_profile_read(jkc_ctx *ctx, int64_t *launches, double *ms);

/* Explicit slice removal of Alg. 2: out = T with slice p of the sampled mode
 * deleted (the reduced tensor of a plain per-submodel fit).  Shapes follow
 * prob (dims of the full tensor); out has dims[sampled_mode]-1 in that mode,
 * same layout rules and dtype as T.  Asynchronous on prob->stream. */
jkc_status jk_cals_remove_slice(const jkc_problem *prob, const void *tensor,
                                int32_t p, void *out);

/* Bytes of the fixed device scratch jk_cals_mttkrp_static works in (one
 * array per GPU the library runs on, held until the process ends). */
#define JKC_STATIC_SCRATCH_BYTES (64ll << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the fused
 * MTTKRP of jk_cals_mttkrp computed from caller buffers without a context or
 * a workspace.  Its scratch -- the other modes' factors padded to the kernel's
 * column pitch (left-out rows of the sampled mode zeroed), the column->model
 * map and left-out row mask, and the split-K partials -- lives in a fixed
 * library-owned device array of JKC_STATIC_SCRATCH_BYTES per GPU; nothing
 * is allocated (no hipMalloc, no allocating library call).
 *   prob    : as for jk_cals_init; precision must be JKC_FP64 (float64
 *             matrix cores), tensor_dtype f64 or f32; copy_tensor and
 *             tree_max_gib are ignored (T is read in place).
 *   tensor  : device, layout above.
 *   factors : host array [N] of device pointers; factors[m] (m != mode) is
 *             I_m x C float64 row-major; factors[mode] is not read (may be
 *             NULL).  The left-out rows of the sampled mode need not be zero.
 *   out     : device I_mode x C float64 row-major; receives T_(mode) times
 *             the multi-factor Khatri-Rao product, the left-out rows of each
 *             model's columns set to 0 when mode is the sampled mode.
 * The same tilings as jk_cals_mttkrp, with at most as many K splits as fit
 * the scratch.  JKC_EINVAL when the padded factors and one output plane need
 * more than JKC_STATIC_SCRATCH_BYTES (the message names both sizes),
 * JKC_EUNSUPPORTED for split precisions.  Asynchronous on prob->stream
 * except for two small table copies from pageable host memory, which finish
 * before the call returns.  Every call on one GPU shares that GPU's scratch:
 * calls that overlap on one GPU (other streams, other threads) race. */
jkc_status jk_cals_mttkrp_static(const jkc_problem *prob, const void *tensor,
                                 const double *const *factors, int32_t mode,
                                 double *out);

/* Free the host-side context (the workspace stays the caller's). */
void jk_cals_destroy(jkc_ctx *ctx);

/* Message for the last non-OK status on this thread ("" if none). */
const char *jk_cals_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* JK_CALS_H */
