/*
 * nmf_beta.h -- C ABI of the MI355X (gfx950) beta-NMF multiplicative-update library.
 *
 * Problem (paper Sec. 2.1, eq. (nmf)): given a nonnegative data matrix V (F x N)
 * and a rank K, find nonnegative W (F x K) and H (K x N) minimizing the separable
 * beta-divergence D_beta(V | WH) = sum_fn d_beta(v_fn | [WH]_fn), eqs. (obj_fct),
 * (beta-div).  With the smoothing constant kappa of Sec. 4.1.3 the objective is
 * D_beta(V + kappa | WH + kappa).
 *
 * Conventions shared by every call:
 *  - Matrices are float32, row-major, in caller-owned DEVICE memory; the leading
 *    dimension (ld*) is the distance in elements between consecutive rows and must
 *    be >= the number of columns.  The library never frees caller memory.
 *  - V is read-only.  W and H are updated in place by nmf_beta_step.
 *  - V, W, H (and dW, dH) must not overlap; overlap is NMF_ERR_ALIAS.
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as void*;
 *    NULL is the null stream).  The returned status covers argument checks and
 *    launch errors only; numeric trouble (a non-finite or zero-denominator update
 *    ratio, a non-finite objective) sets sticky device flags read by nmf_get_flags.
 *  - Device scalars (double* d_objective ...) are caller-owned device memory.
 *  - A context owns a workspace on one device.  It grows on demand (a blocking
 *    reallocation) until the first call recorded into a stream capture.  From
 *    then on it never moves, since a captured graph may point into it: a call
 *    (captured or not, nmf_reserve included) that needs a larger workspace
 *    returns NMF_ERR_WORKSPACE.  Call nmf_reserve first to size it once for
 *    every shape a graph will use; use another context for larger shapes.
 *  - A context must not be used by two host threads at the same time, and two
 *    calls on different streams through one context must not overlap in time
 *    (they share the workspace).
 *  - Supported sizes: F, N >= 1, 1 <= K <= 128.
 */
#ifndef NMF_BETA_H
#define NMF_BETA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmf_ctx_s* nmf_ctx_t;

typedef enum {
  NMF_OK = 0,
  NMF_ERR_NULL = 1,        /* a required pointer is NULL */
  NMF_ERR_SHAPE = 2,       /* F, N or K < 1, or a leading dimension too small */
  NMF_ERR_BETA = 3,        /* beta or kappa not finite, kappa < 0 */
  NMF_ERR_ALIAS = 4,       /* two of the matrices overlap in memory */
  NMF_ERR_WORKSPACE = 5,   /* workspace too small while the stream is captured, or
                              after a call was captured (the workspace no longer moves) */
  NMF_ERR_HIP = 6,         /* a HIP runtime call failed */
  NMF_ERR_UNSUPPORTED = 7, /* K > 128, unknown precision, an unsupported inner_iters > 1 case */
  NMF_ERR_ARG = 8,         /* other invalid argument (mode, opts field) */
  NMF_ERR_NO_DEVICE = 9,   /* no usable GPU */
  NMF_ERR_IO = 10          /* nmf_tune could not write its cache file */
} nmf_status;

typedef enum {
  NMF_ALTERNATING = 0, /* block MM, Sec. 2.2 eq. (alt_update), Algorithm 1 */
  NMF_JOINT = 1        /* joint MM, Sec. 3.2 eq. (jnt_update), Algorithm 2 */
} nmf_mode;

typedef enum {
  NMF_FP32 = 0, /* every product in float32 (matrix cores, fp32 accumulate) */
  NMF_BF16 = 1, /* products on bfloat16 matrix cores, fp32 accumulate: the W- and
                   H-step contractions with single bfloat16 operands; Lambda = WH
                   as hi*hi + lo*hi + hi*lo of split operands (about 2^-16
                   relative), so the float32 element-wise terms and the float64
                   objective see an almost float32 Lambda.  K <= 64. */
  NMF_FP16 = 2  /* the same with float16 operands (operands must stay within
                   float16 range).  K <= 64. */
} nmf_precision;

/* sticky numeric flags (nmf_get_flags) */
#define NMF_FLAG_NONFINITE 1u /* an update ratio num/den was non-finite or den <= 0 */
#define NMF_FLAG_DOMAIN 2u    /* nmf_beta_validate found data outside the domain */
#define NMF_FLAG_BARRIER 4u   /* a batched step's work item gave up waiting for its
                                 problem's previous phase (bounded poll); the results
                                 of that launch are invalid.  The single-launch path
                                 synchronizes with cooperative grid barriers, which
                                 do not give up, and never sets it. */
#define NMF_FLAG_RANGE 8u     /* NMF_FP16 mode: an operand of a float16 product was
                                 outside the float16 range or not finite (the step's
                                 result is then not meaningful) */
#define NMF_FLAG_SKIPPED 16u  /* nmf_beta_step_batched updated nothing: a descriptor
                                 was invalid, two problems' matrices overlapped, or
                                 the batch needed more than the reserved region */

/* exponent of the multiplicative updates (nmf_step_opts.exponent) */
#define NMF_EXPONENT_MM 0  /* gamma(beta) of eq. (def_gamma): the MM step, whose
                              objective never increases */
#define NMF_EXPONENT_ONE 1 /* 1 for every beta: the heuristic discussed for both
                              methods in Sec. 3.3.3 ("Failure of heuristic
                              updates"); outside 1 <= beta <= 2 it is not an MM
                              step, and the objective may increase */

typedef struct {
  int32_t precision;   /* nmf_precision; default NMF_FP32 */
  float kappa;         /* smoothing constant of Sec. 4.1.3, >= 0; default 0 */
  int32_t inner_iters; /* sub-iterations L (1 <= L <= 1000; else NMF_ERR_ARG).
                          NMF_ALTERNATING (Algorithm 1): L W updates, each against
                          the latest W, then L H updates against the final W.
                          NMF_JOINT (Algorithm 2): L alternations of a W and an H
                          update, both always multiplying the tilde iterate, with
                          V~, P, Q formed once (F N <= 2^28, NMF_FP32).  L > 1
                          is not available in batches or on the single-launch
                          path (NMF_ERR_UNSUPPORTED); default 1 */
  int32_t normalize;   /* 1: divide W's columns by their l2 norm and scale H's rows
                          (Sec. 4.1.2) at the end of the step; default 1 */
  int32_t exponent;    /* NMF_EXPONENT_MM (default) or NMF_EXPONENT_ONE; other
                          values: NMF_ERR_ARG */
  int32_t gram;        /* 1: at beta = 2, the denominators in the Gram form of
                          Table 2 (Sec. 3.3.1): Q H~^T = W~ (H~ H~^T) and
                          chi_2^T Q = (chi_2^T W~) H~ (joint; W_new^T W_new H~
                          alternating), with the K x K products formed in float64,
                          so both passes over V contract P = V only and the H pass
                          forms no Lambda.  Needs beta = 2, kappa = 0, NMF_FP32,
                          inner_iters = 1, K <= 64 (else NMF_ERR_UNSUPPORTED); not
                          in batches.  0 (default): the contraction form. */
} nmf_step_opts;

/* Fills *opts with the defaults listed above. */
void nmf_default_opts(nmf_step_opts* opts);

/* Library version string (static storage). */
const char* nmf_version(void);

/* Human-readable name of a status code (static storage, never NULL). */
const char* nmf_status_string(nmf_status status);

/* Creates a context on HIP device `device`.  No workspace is allocated yet.
 * NMF_ERR_NO_DEVICE if the device does not exist.  *out is NULL on error. */
nmf_status nmf_create(nmf_ctx_t* out, int device);

/* Releases the context and its workspace (synchronizes the device first). */
nmf_status nmf_destroy(nmf_ctx_t ctx);

/* Sizes the workspace for every later call with F <= maxF, N <= maxN, K <= maxK,
 * so that those calls never allocate (required before stream capture). */
nmf_status nmf_reserve(nmf_ctx_t ctx, int64_t maxF, int64_t maxN, int64_t maxK);

/* Host-only argument check of nmf_beta_step (no HIP call, usable without a GPU).
 * Returns the status nmf_beta_step would return for these arguments before any
 * device work.  opts may be NULL (defaults). */
nmf_status nmf_check_step_args(int64_t F, int64_t N, int64_t K, const float* V, int64_t ldv,
                               const float* W, int64_t ldw, const float* H, int64_t ldh,
                               double beta, int32_t mode, const nmf_step_opts* opts);

/* One outer iteration of the multiplicative-update method, in place on W and H.
 *
 * mode == NMF_ALTERNATING (paper Sec. 2.2, eq. (alt_update), Algorithm 1 with
 *   L_W = L_H = opts->inner_iters, default 1):
 *   W <- W .* ((( (WH)^(b-2) .* V) H^T) / ((WH)^(b-1) H^T))^gamma,
 *   then H is updated the same way against the new W (WH is formed again).
 * mode == NMF_JOINT (paper Sec. 3.2, eq. (jnt_update), Algorithm 2 with
 *   L = opts->inner_iters, default 1): V~ = W~H~ is formed once; W and H are
 *   both updated from the tilde iterate, the H step using chi_1(W, W~) and
 *   chi_2(W, W~) in its contractions (and, for L > 1, the W step chi_1(H, H~)
 *   and chi_2(H, H~)).
 * gamma = gamma(beta) of eq. (def_gamma), or 1 with opts->exponent ==
 * NMF_EXPONENT_ONE.  With opts->normalize the columns of W
 * are scaled to unit l2 norm and the rows of H by the inverse (Sec. 4.1.2).
 * At L = 1 the W step of both modes is the same computation (Sec. 4.1.1).
 *
 * d_objective (device double, may be NULL) receives D_beta(V + kappa | W~H~ + kappa)
 * at the ENTRY iterate, computed in the same pass over V.
 */
nmf_status nmf_beta_step(nmf_ctx_t ctx, void* stream, int64_t F, int64_t N, int64_t K,
                         const float* V, int64_t ldv, float* W, int64_t ldw, float* H, int64_t ldh,
                         double beta, int32_t mode, const nmf_step_opts* opts, double* d_objective);

/* nmf_beta_step for callers that cannot allocate device memory: code under
 * HIP graph capture without a prior nmf_reserve, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same arguments, semantics and results as
 * nmf_beta_step (the same kernels and launch plan), plus d_flags.
 *
 * Workspace: a fixed array of NMF_NOALLOC_SCRATCH_BYTES per GPU, part of the
 * library's code object (held from the library's first use on a device until
 * the process ends); this call allocates and frees nothing.  A step whose
 * workspace does not fit returns NMF_ERR_WORKSPACE before any device work.
 * The joint step keeps its P, Q tiles between the passes only when they fit as
 * well (otherwise its H pass forms V~ again, as above 2^28 entries); joint
 * sub-iterations (inner_iters > 1) need the kept tiles.  At K = 64 (float32)
 * the joint step keeps them up to about 4M entries of V (1024 x 4096: 81 MiB),
 * and without them both modes fit beyond 4096 x 4096 (69 MiB); the partial
 * sums of the split reductions and the F x K terms set the limit.  The
 * single-launch path (nmf_set_path) and kernel timing (nmf_profile_enable)
 * are not used.
 *
 * Every call on one GPU shares that GPU's array: two calls that overlap in time
 * on one GPU (different streams, contexts or host threads) race and give
 * undefined results.  Each call writes every part of the array it reads, so
 * nothing needs clearing between calls.
 *
 * d_flags (device uint32, nullable): the sticky NMF_FLAG_* bits of this call
 * are OR-ed into it (the caller clears it); with NULL they are discarded.
 * nmf_get_flags does not see them. */
#define NMF_NOALLOC_SCRATCH_BYTES (96u << 20)
nmf_status nmf_beta_step_noalloc(nmf_ctx_t ctx, void* stream, int64_t F, int64_t N, int64_t K,
                                 const float* V, int64_t ldv, float* W, int64_t ldw, float* H,
                                 int64_t ldh, double beta, int32_t mode, const nmf_step_opts* opts,
                                 double* d_objective, uint32_t* d_flags);

/* D_beta(V + kappa | WH + kappa) (eqs. (obj_fct), (beta-div)) written to the device
 * double *d_out.  Per-entry terms and the reduction are float64; WH is float32.
 * At v = 0 the limit is used (beta = 1: the term is [WH]_fn; beta <= 0: +inf). */
nmf_status nmf_beta_objective(nmf_ctx_t ctx, void* stream, int64_t F, int64_t N, int64_t K,
                              const float* V, int64_t ldv, const float* W, int64_t ldw,
                              const float* H, int64_t ldh, double beta, float kappa, double* d_out);

/* Gradient of D_beta(V + kappa | WH + kappa) w.r.t. W and H, times `scale` and,
 * when d_scale (a device double) is not NULL, times *d_scale read on the device
 * (so an upstream gradient that lives on the device needs no host sync):
 *   E = (WH + kappa)^(beta-2) .* (WH - V),  dW = s * E H^T,  dH = s * W^T E.
 * (E is the derivative of d_beta in its second argument; these are the bracketed
 * terms of the KKT residuals of Sec. 4.1.5.)  dW is F x K (ld lddw), dH is K x N
 * (ld lddh), both caller-owned device float32.  d_objective (nullable) receives
 * the objective at (W, H).  No gradient w.r.t. V is computed. */
nmf_status nmf_beta_grad(nmf_ctx_t ctx, void* stream, int64_t F, int64_t N, int64_t K,
                         const float* V, int64_t ldv, const float* W, int64_t ldw,
                         const float* H, int64_t ldh, double beta, float kappa, double scale,
                         const double* d_scale, float* dW, int64_t lddw, float* dH, int64_t lddh,
                         double* d_objective);

/* KKT residuals of Sec. 4.1.5 at (W, H), written to the device doubles
 * d_res[0] = || min(W, grad_W D) ||_1 / (F K) and d_res[1] = || min(H, grad_H D) ||_1 / (K N),
 * with D = D_beta(V + kappa | WH + kappa) and the gradients of nmf_beta_grad
 * (float32 passes, float64 minimum, absolute value and sums). */
nmf_status nmf_beta_kkt(nmf_ctx_t ctx, void* stream, int64_t F, int64_t N, int64_t K,
                        const float* V, int64_t ldv, const float* W, int64_t ldw,
                        const float* H, int64_t ldh, double beta, float kappa, double* d_res);

/* Up to max_iters outer iterations (nmf_beta_step with these mode and opts) with
 * the stopping rule of Sec. 4.1.2 evaluated on the device, so that the whole
 * run can be captured in one graph and needs no host synchronization:
 *   d_trace[t] = D_beta(V + kappa | W_t H_t + kappa) of iterate t (t = 0 the
 *   caller's W, H), formed in iterate t's own pass over V;
 *   the run stops at the first t >= 1 with (d_trace[t-1] - d_trace[t]) / d_trace[t]
 *   <= eps (as printed, no absolute value; the paper uses eps = 1e-5): W, H then
 *   hold iterate t, *d_stop = t, and d_trace[t+1 ..] are not written.  Without a
 *   stop, W, H hold iterate max_iters, d_trace[max_iters] its objective, and
 *   *d_stop = -1.
 * Every launch after the stop does nothing (each kernel reads the halt word).
 * d_trace (device double[max_iters + 1]) and d_stop (device int32) are caller
 * memory.  The single-launch path is not used.  max_iters >= 0. */
nmf_status nmf_beta_run(nmf_ctx_t ctx, void* stream, int64_t F, int64_t N, int64_t K,
                        const float* V, int64_t ldv, float* W, int64_t ldw, float* H, int64_t ldh,
                        double beta, int32_t mode, const nmf_step_opts* opts, int32_t max_iters,
                        double eps, double* d_trace, int32_t* d_stop);

/* Scans V, W, H once and sets NMF_FLAG_DOMAIN if V has a negative or non-finite
 * entry, W or H a non-positive or non-finite entry, or (beta <= 0, kappa == 0) V
 * has a zero (where d_beta is infinite, Sec. 4.1.3). */
nmf_status nmf_beta_validate(nmf_ctx_t ctx, void* stream, int64_t F, int64_t N, int64_t K,
                             const float* V, int64_t ldv, const float* W, int64_t ldw,
                             const float* H, int64_t ldh, double beta, float kappa);

/* Reads (synchronizing `stream`) and optionally clears the sticky flags: those of
 * the context's steps and of its nmf_beta_step_batched calls, OR-ed together. */
nmf_status nmf_get_flags(nmf_ctx_t ctx, void* stream, uint32_t* flags, int32_t clear);

/* Per-kernel timing with HIP events recorded on the launch stream around each
 * launch of the selected kernels (bit mask of NMF_KERNEL_* values; 0 disables).
 * nmf_profile_read synchronizes the recorded events and returns the summed
 * duration in milliseconds and the number of timed launches of one kernel since
 * the last reset, then resets that kernel's counters. */
#define NMF_KERNEL_SWEEP_W 0   /* pass over V accumulating the W-step contractions */
#define NMF_KERNEL_UPDATE_W 1  /* reduction of W partials, W update, chi terms */
#define NMF_KERNEL_SWEEP_H 2   /* pass over V accumulating the H-step contractions */
#define NMF_KERNEL_UPDATE_H 3  /* reduction of H partials, H update, normalization */
#define NMF_KERNEL_FUSED_STEP 5 /* whole outer iteration in one cooperative launch */
#define NMF_KERNEL_SPARSE_PASS 6 /* sparse beta = 1 step: row pass (+ column pass in joint mode) */
#define NMF_KERNEL_SPARSE_COLS 7 /* sparse beta = 1 step, alternating mode: column pass */
#define NMF_KERNEL_COUNT 8
nmf_status nmf_profile_enable(nmf_ctx_t ctx, uint32_t kernel_mask);
/* With NMF_KERNEL_FUSED_STEP selected, the single-launch step also records the
 * device clock at its phase boundaries; this returns (synchronizing `stream`)
 * the n <= 7 intervals of the most recent launch in microseconds: W pass, grid
 * barrier, W update, barrier, H pass, barrier, H update. */
nmf_status nmf_profile_phases(nmf_ctx_t ctx, void* stream, double* us, int32_t n);
nmf_status nmf_profile_read(nmf_ctx_t ctx, int32_t kernel, double* total_ms, int64_t* launches);

/* Execution path of nmf_beta_step.  STREAM: four launches per outer iteration
 * (W pass, W update, H pass, H update).  FUSED: one cooperative launch running
 * the same four phases separated by grid barriers; in joint mode its H pass
 * contracts the element-wise terms P, Q stored by the W pass instead of forming
 * Lambda again; available for F*N <= 2^24 and K <= 64 outside stream capture,
 * else NMF_ERR_UNSUPPORTED.  AUTO (default) currently selects STREAM, the
 * faster of the two on MI355X at every size measured.  Results agree to
 * rounding between the paths. */
#define NMF_PATH_AUTO 0
#define NMF_PATH_STREAM 1
#define NMF_PATH_FUSED 2
nmf_status nmf_set_path(nmf_ctx_t ctx, int32_t path);

/* Launch geometry override for tuning: target number of workgroups per sweep
 * (0 = default, twice the number of compute units) and minimum number of 32-wide
 * tiles each workgroup walks (0 = default 1).  Applies to later calls. */
nmf_status nmf_set_launch(nmf_ctx_t ctx, int32_t target_blocks, int32_t min_tiles);

/* ---------------------------------------------------------------------------
 * beta = 1 (Kullback-Leibler) with a sparse V.
 *
 * For count data most of V is zero (the play counts of Sec. 4.4 are about 0.6 %
 * nonzero).  At beta = 1 the updates of Table 2 (Sec. 3.3.1) need V / (WH)
 * only where v != 0, and their denominators are row sums of H~ and column
 * sums of W_new, so a step touches only the nonzeros:
 *   W step:                numW = P H~^T, P = V / (W~ H~) at the nonzeros,
 *                          denW = row sums of H~;
 *   H step, NMF_JOINT:     numH = W~^T P with the same P (chi_1 = W~ at beta = 1),
 *                          denH = column sums of W_new (chi_2 = W_new);
 *   H step, NMF_ALTERNATING: numH = W_new^T P', P' = V / (W_new H~), same denH.
 * D_1(V | WH) = sum of all [WH]_fn (from factor sums) + sum over the nonzeros
 * of v log(v / [WH]_fn) - v.  An entry with v = 0 never evaluates V / (WH)
 * (a row of V without nonzeros gives a zero row of W_new, with no 0/0).
 *
 * V is given by its nonzeros twice, in caller-owned device memory: row order
 * (CSR) and column order (CSC) of the same entries.  Columns (rows) must
 * ascend within a row (column).  The library reads the indices clamped to the
 * matrix and the pointers clamped to [0, nnz], so a malformed matrix gives
 * wrong numbers but no access outside the arrays; nmf_sparse_validate checks
 * the structure.  F, N >= 1, nnz >= 0, 1 <= K <= 64, float32 products only,
 * kappa = 0 (V + kappa would be dense), inner_iters = 1 (else
 * NMF_ERR_UNSUPPORTED).  gamma(1) = 1, so opts->exponent changes nothing.
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t F, N, nnz;
  const int64_t* row_ptr;  /* [F + 1]: entries of row f are row_ptr[f] .. row_ptr[f + 1] - 1 */
  const int32_t* col_idx;  /* [nnz]: column of each entry, in row order */
  const float* row_val;    /* [nnz]: value of each entry, in row order (>= 0) */
  const int64_t* col_ptr;  /* [N + 1]: entries of column n, in column order */
  const int32_t* row_idx;  /* [nnz]: row of each entry, in column order */
  const float* col_val;    /* [nnz]: the same values, in column order */
} nmf_sparse_v;

/* One outer iteration at beta = 1 on a sparse V, in place on W (F x K, ld ldw)
 * and H (K x N, ld ldh); mode NMF_JOINT or NMF_ALTERNATING; opts as for
 * nmf_beta_step within the limits above (normalize is honoured).  d_objective
 * (device double, nullable) receives D_1(V | W~H~) of the entry iterate. */
nmf_status nmf_kl_step_sparse(nmf_ctx_t ctx, void* stream, const nmf_sparse_v* V, int64_t K, float* W,
                              int64_t ldw, float* H, int64_t ldh, int32_t mode,
                              const nmf_step_opts* opts, double* d_objective);

/* D_1(V | WH) for a sparse V, written to the device double *d_out. */
nmf_status nmf_kl_objective_sparse(nmf_ctx_t ctx, void* stream, const nmf_sparse_v* V, int64_t K,
                                   const float* W, int64_t ldw, const float* H, int64_t ldh,
                                   double* d_out);

/* Scans both orders of a sparse V and sets NMF_FLAG_DOMAIN when a pointer array
 * does not start at 0, end at nnz and never decrease, an index is out of range
 * or not ascending within its row (column), or a value is negative or not
 * finite. */
nmf_status nmf_sparse_validate(nmf_ctx_t ctx, void* stream, const nmf_sparse_v* V);

/* ---------------------------------------------------------------------------
 * Many problems in one launch.
 *
 * A batch holds P independent problems of uneven sizes, each with its own beta
 * (and K <= 64), and runs one outer iteration of every problem -- the same
 * computation as nmf_beta_step in the batch's mode -- in ONE persistent kernel
 * launch.  Work items of all problems (W pass, W update, H pass, H update) are
 * taken from a queue listed phase by phase; a per-problem completion counter
 * lets an item start once its problem's previous phase that has items has
 * finished.  A problem whose rows take one column group has no W-update items
 * (its W-pass items apply the W update), and if its columns also take one row
 * group no H-update items either (its H-pass items apply the H update).
 *
 * The batch owns its own device memory (descriptors, queue, workspace, status
 * word), allocated by nmf_batch_create; nmf_batch_step allocates nothing and
 * may be captured into a HIP graph.  The problems' V, W, H stay caller-owned;
 * their pointers are fixed at creation.  W and H of different problems must not
 * overlap each other or any V (NMF_ERR_ALIAS); V may be shared.
 * ------------------------------------------------------------------------- */
typedef struct nmf_batch_s* nmf_batch_t;

typedef struct {
  int64_t F, N, K;          /* sizes; 1 <= K <= 64 */
  const float* V; int64_t ldv;
  float* W; int64_t ldw;
  float* H; int64_t ldh;
  double beta;
} nmf_problem;

typedef struct {
  int32_t tiles_per_item;   /* 32-wide tiles each pass item walks (0: the context's
                               per-bucket table, 256 in every bucket unless set by
                               nmf_set_batch_tiles or nmf_tune) */
  int32_t workers;          /* persistent workgroups (0: as many as fit on the GPU) */
  int32_t lag;              /* order of the work queue.  0 (default): phase by phase
                               over all problems.  d > 0: problems pipelined d apart,
                               problem j's phase q listed with problem j + q d's W
                               pass, so a problem's kept P, Q are read back by its H
                               pass while fewer problems' tiles are in flight. */
} nmf_batch_config;

/* Validates every problem (as nmf_beta_step would; opts->precision FP32 or BF16,
 * inner_iters 1), plans the work items, allocates and uploads the batch.  `cfg`
 * may be NULL (defaults).  Synchronous.  *out is NULL on error. */
nmf_status nmf_batch_create(nmf_ctx_t ctx, const nmf_problem* problems, int32_t count, int32_t mode,
                            const nmf_step_opts* opts, const nmf_batch_config* cfg, nmf_batch_t* out);

/* One outer iteration of every problem in one launch on `stream`.
 * d_objectives (device double[count], may be NULL) receives each problem's
 * objective at its entry iterate. */
nmf_status nmf_batch_step(nmf_batch_t batch, void* stream, double* d_objectives);

/* Sticky flags of the batch (as nmf_get_flags); NMF_FLAG_BARRIER means a work
 * item gave up waiting for its problem's previous phase. */
nmf_status nmf_batch_get_flags(nmf_batch_t batch, void* stream, uint32_t* flags, int32_t clear);

/* Number of work items per launch and persistent workgroups of the batch. */
nmf_status nmf_batch_info(nmf_batch_t batch, int64_t* work_items, int32_t* workers, int64_t* device_bytes);

/* Frees the batch (synchronizes the device first). */
nmf_status nmf_batch_destroy(nmf_batch_t batch);

/* Per-bucket tile counts.  A problem of a batch falls in bucket
 *   6 (4 k + s) + c,
 *   k = (K <= 32 ? 0 : 1),
 *   s = (T <= 32 ? 0 : T <= 64 ? 1 : T <= 128 ? 2 : 3), T = max(ceil(F / 32), ceil(N / 32)),
 *   c = the beta class: 0 general, 1 beta = 2, 2 beta = 1, 3 beta = 0, 4 beta = 1/2,
 *       5 beta = 3/2 (the classes the kernels are compiled for),
 * and walks the tiles_per_item of its bucket.  The context holds one table
 * (256 in every bucket at creation), used by nmf_batch_create when
 * cfg->tiles_per_item is 0 and by every nmf_beta_step_batched. */
#define NMF_BATCH_BUCKETS 48

/* Bucket of a problem of sizes F, N, K and divergence beta (host only); -1 if
 * a size is out of range (F, N < 1, K outside 1..64) or beta is not finite. */
int32_t nmf_batch_bucket(int64_t F, int64_t N, int64_t K, double beta);

/* Sets (copies in) or reads (copies out) the context's table of
 * NMF_BATCH_BUCKETS tile counts, each in 1..4096 (else NMF_ERR_ARG).  Setting
 * also updates the reserved batched region if there is one (a blocking copy):
 * graphs that replay nmf_beta_step_batched plan with the new table from their
 * next replay on. */
nmf_status nmf_set_batch_tiles(nmf_ctx_t ctx, const int32_t* tiles);
nmf_status nmf_get_batch_tiles(nmf_ctx_t ctx, int32_t* tiles);

/* Autotuner of the context's bucket table for a representative set of
 * problems (host descriptors of device matrices, as nmf_batch_create).
 *
 * Key: the device's architecture and compute-unit count, the mode and
 * opts->precision.  If `cache_path` (may be NULL) holds an entry for this key
 * that covers every bucket the problems fall in, its tiles are installed and
 * nothing is measured (*from_cache = 1).  Otherwise, starting from that entry
 * (else from the context's table), each uncovered bucket in turn takes the
 * candidate of {4, 8, 16, 32, 64, 128, 256} with the smallest time per batched step
 * of the whole set (one warm-up step, then `iters` timed steps; candidates
 * that split every problem of the bucket as an already timed one are skipped),
 * the others held fixed.  The problems' W and H are saved before and restored
 * after every timing, so they are unchanged on return.  The result is
 * installed in the context (as nmf_set_batch_tiles) and, with a cache_path,
 * written to the file (one text line per key, other lines kept; written to a
 * temporary file and renamed; NMF_ERR_IO if that fails).
 *
 * tiles (host int32[NMF_BATCH_BUCKETS], required) receives the table; ms
 * (nullable) the time per step of the set with it (the cached time on a cache
 * hit); from_cache (nullable) 1 on a cache hit, else 0.  Synchronous; not
 * during stream capture. */
nmf_status nmf_tune(nmf_ctx_t ctx, void* stream, const nmf_problem* problems, int32_t count, int32_t mode,
                    const nmf_step_opts* opts, int32_t iters, const char* cache_path, int32_t* tiles, double* ms,
                    int32_t* from_cache);

/* ---------------------------------------------------------------------------
 * Batched step with descriptors in device memory.
 *
 * For callers whose problem set changes between steps without a host round
 * trip: a graph replayed over new matrices, shapes or betas, or a serving loop
 * that cannot call hipMalloc.  nmf_reserve_batched sizes the context's batched
 * region once; nmf_beta_step_batched then allocates nothing and never waits on
 * the host, so it may be captured into a HIP graph.  Each call launches a
 * planning kernel (one workgroup: it reads the descriptors, checks them, plans
 * every problem with the context's bucket table exactly as nmf_batch_create
 * does, lays the workspaces out, and lists the work items phase by phase,
 * larger problems first) and then the persistent kernel of nmf_batch_step.  The
 * results are those of nmf_batch_create + nmf_batch_step on the same problems
 * with the same tile counts and lag 0.
 * ------------------------------------------------------------------------- */

/* Items per step and workspace bytes that `count` problems (host descriptors;
 * only the sizes and beta are read) need in `mode` and `precision` (NMF_FP32 or
 * NMF_BF16) under `tiles` (host int32[NMF_BATCH_BUCKETS]; NULL: 256 in every
 * bucket).  The item count is the batch's exact one: a problem whose rows take
 * one column group has its W update applied by its W-pass items (no W-update
 * items), and if its columns also take one row group its H update by its
 * H-pass items (no H-update items).  Host only, no GPU.  NMF_ERR_ARG for a bad
 * mode, precision or table, NMF_ERR_UNSUPPORTED for NMF_FP16 or K > 64,
 * NMF_ERR_SHAPE for a size out of range, NMF_ERR_BETA for a beta that is not
 * finite. */
nmf_status nmf_batch_requirements(const nmf_problem* problems, int32_t count, int32_t mode, int32_t precision,
                                  const int32_t* tiles, int64_t* items, int64_t* workspace_bytes);

/* Allocates the context's batched region (blocking; frees a previous one):
 * max_problems descriptors (>= 1), max_items work items per step (1 .. 2^31 - 1)
 * and workspace_bytes (>= 0) of problem workspaces.  NMF_ERR_WORKSPACE once a
 * nmf_beta_step_batched call was captured (a graph may point into the region). */
nmf_status nmf_reserve_batched(nmf_ctx_t ctx, int32_t max_problems, int64_t max_items, int64_t workspace_bytes);

/* One outer iteration of every problem described by d_problems (device array
 * of `count` nmf_problem, count <= max_problems), in place on their W and H.
 * d_count (device int32, nullable): the number of descriptors used this call,
 * read on the device (0 <= *d_count <= count), so a captured call can be
 * replayed on fewer problems; NULL uses all `count`.  opts: FP32 or BF16,
 * inner_iters 1, gram 0 (else NMF_ERR_UNSUPPORTED).  d_objectives (device
 * double[count], nullable) receives each problem's entry objective.
 *
 * Status covers the host arguments: NMF_ERR_NULL, NMF_ERR_ARG (count < 1, mode,
 * opts), NMF_ERR_WORKSPACE (no batched region, or count > max_problems).  The
 * descriptors are checked on the device (as nmf_beta_step's arguments, K <= 64,
 * and the W and H of every problem overlapping no other W, H and no V; V may
 * be shared):
 * if one fails, or the plan needs more items or workspace than reserved, the
 * call updates nothing, writes no objective and sets NMF_FLAG_SKIPPED.  Flags
 * of these calls are read and cleared with nmf_get_flags.  Calls on one
 * context share the region: calls that overlap in time race. */
nmf_status nmf_beta_step_batched(nmf_ctx_t ctx, void* stream, int32_t count, const nmf_problem* d_problems,
                                 int32_t mode, const nmf_step_opts* opts, double* d_objectives,
                                 const int32_t* d_count);

#ifdef __cplusplus
}
#endif
#endif /* NMF_BETA_H */
