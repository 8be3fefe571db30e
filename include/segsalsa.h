/*
 * segsalsa.h -- C ABI of the MI355X (gfx950) SegSALSA-STR solver.
 *
 * SegSALSA-STR (Condessa, Bioucas-Dias, Kovacevic, arXiv 1504.07028) computes
 * the marginal-MAP hidden field z in R^{K x n} of a segmentation problem,
 *
 *     min_z  sum_i -ln(p_i^T z_i) + lambda sum_i ||[J z]_i||_{S_p}       (eq. (7))
 *     s.t.   z >= 0,  1_K^T z_i = 1,
 *
 * where J is the patch-based Jacobian of eq. (4), by the SALSA iteration of
 * eqs. (12)-(14) applied to the four-term splitting of eqs. (8)-(11).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arrays are class-planar and row-major: element (k, r, c) of a [K][H][W]
 *    array is at k*H*W + r*W + c.  Pixel i = r*W + c.
 *  - Pointers are DEVICE pointers owned by the caller unless marked HOST.
 *    The library allocates no device memory: every call takes a caller
 *    workspace whose size comes from the matching *_workspace_size query.
 *  - `precision` selects the element type of every floating-point array:
 *    float for SEGSALSA_FP32, double for SEGSALSA_FP64.
 *  - Argument errors are detected on the host before anything is enqueued
 *    and returned as a status; the thread-local message is available from
 *    segsalsa_last_error().  Work is enqueued asynchronously on `stream`
 *    (a hipStream_t; NULL is the default stream).  A call that is given a
 *    HOST stats pointer waits for the stream before it returns.
 *  - No C++ exception crosses this interface.
 *
 * Readings of the paper used throughout (the paper is silent or ambiguous):
 *  - initialisation z^0 = p_i / 1^T p_i (or softmax of logits), all scaled
 *    multipliers d = 0, u^0 = G z^0;
 *  - one round = u-update (eq. (13), at the z of the latest z-update) ->
 *    d-update (eq. (14)) -> z-update (eq. (12)); `iters` rounds return the
 *    paper's z^{iters+1};
 *  - D_h, D_v are forward differences with periodic boundaries; P_j shifts
 *    by the j-th patch offset (dy, dx) in row-major order (dy outer) and
 *    scales by the caller's multiplier c_j;
 *  - g4 is the indicator of {1_K^T xi = 1} (eq. (10)): its proximity
 *    operator is the affine projection; positivity comes from g3
 *    (g4_simplex = 1 selects the simplex projection of Sec. 4's wording).
 */
#ifndef SEGSALSA_H
#define SEGSALSA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SEGSALSA_OK = 0,
  SEGSALSA_ERR_INVALID_ARG = 1,  /* a size, pointer or parameter is out of range        */
  SEGSALSA_ERR_UNSUPPORTED = 2,  /* valid for the method but not implemented here       */
  SEGSALSA_ERR_WORKSPACE = 3,    /* workspace NULL, misaligned or smaller than required */
  SEGSALSA_ERR_DEVICE = 4        /* a HIP call failed (message in segsalsa_last_error)  */
} segsalsa_status;

typedef enum { SEGSALSA_FP32 = 0, SEGSALSA_FP64 = 1 } segsalsa_precision;

/* Flags reported in segsalsa_stats.flags (set by the device-side input check). */
#define SEGSALSA_FLAG_NONFINITE_INPUT 1   /* an input value is NaN or infinite          */
#define SEGSALSA_FLAG_NEGATIVE_PROB 2     /* a probability is negative                  */
#define SEGSALSA_FLAG_ZERO_PIXEL 4        /* a pixel's probabilities sum to 0            */

/* One problem of eq. (7) and its SALSA parameters. */
typedef struct {
  int32_t K;                   /* classes, 2 <= K <= 64; each workgroup keeps every class of its
                                  pixels in registers, so larger patches allow fewer classes
                                  (else UNSUPPORTED): FP32 K <= 64 for M <= 1, 32 for M = 2,
                                  16 for M >= 3; FP64 K <= 64 for M = 0, 32 for M = 1, 16 for
                                  M >= 2                                                          */
  int32_t H, W;                /* image rows and columns, 1 <= H, W <= 4096, H*W >= 2           */
  int32_t patch_radius;        /* M in [0, 5]: (2M+1) x (2M+1) patch, L = (2M+1)^2 (Sec. 3)     */
  const double *patch_weights; /* HOST, L finite multipliers c_j of P_j (eq. (4)), row-major in
                                  (dy, dx) with dy outer; not all zero                            */
  double schatten_p;           /* p >= 1 or INFINITY (the Schatten norm of Sec. 3): 1, 2 and inf
                                  in closed form, other p by a per-pixel Newton solve of the
                                  shrunk singular-value pair; p < 1 or NaN -> INVALID_ARG          */
  double lambda;               /* prior weight of eq. (6), finite, >= 0                          */
  double mu;                   /* SALSA penalty of eq. (13), finite, > 0                          */
  int32_t iters;               /* rounds, >= 0                                                    */
  int32_t input_is_logits;     /* 0: input holds probabilities (>= 0, finite, positive sum per
                                  pixel); 1: input holds logits and p = softmax over classes      */
  int32_t residual_every;      /* > 0: compute the primal and dual residuals after every
                                  residual_every-th round and after the last one, report the last
                                  ones and the objective in stats (needs a HOST stats pointer);
                                  each checked round waits for the stream.  Checked rounds run a
                                  build of the proximity kernel that also sums the residuals, so
                                  their rounding may differ from unchecked rounds in the last bit */
  double tol;                  /* > 0: stop after the first checked round whose primal and dual
                                  residuals are both <= tol (the paper's stopping rule, Sec. 4);
                                  needs residual_every > 0.  0: run exactly `iters` rounds        */
  int32_t warm_start;          /* 0: initialise the state from the input.  1: continue from the
                                  state already in the workspace and z_out, left there by an
                                  earlier call with the same problem, precision and workspace     */
  int32_t use_graph;           /* 1: capture the whole solve (set-up, initialisation, all rounds)
                                  into a hipGraph on first use and replay it on later calls with
                                  the same problem, buffers and workspace (one graph launch per
                                  call; cannot be combined with residual_every).  0: launch the
                                  kernels directly                                               */
  int32_t g4_simplex;          /* reading of the fourth split g4 (eq. (10) vs Sec. 4's wording):
                                  0: projection onto {1_K^T xi = 1} (the definition); 1: projection
                                  onto the probability simplex (Sec. 4's text).  Both reach the
                                  same minimiser with g3; their iterates differ                   */
} segsalsa_problem;

/* Results reported to a HOST stats pointer. */
typedef struct {
  double primal_res;   /* ||G z - u||_F of the last checked round (0 if never checked)        */
  double dual_res;     /* mu ||G (z_new - z_old)||_F of the last checked round                */
  double objective;    /* eq. (7) at the projection of z onto the simplex, with the input's
                          normalised p (computed when residual_every > 0, else 0)            */
  int32_t rounds_done; /* rounds executed by this call                                       */
  int32_t flags;       /* SEGSALSA_FLAG_* bits from the input check of the initialisation    */
} segsalsa_stats;

/* Human-readable name of a status code (static string). */
const char *segsalsa_status_string(segsalsa_status s);

/* Message describing the last error returned on the calling thread ("" if none). */
const char *segsalsa_last_error(void);

/*
 * Bytes of device workspace that segsalsa_str_solve needs for `prob` at
 * `precision`.  Depends only on K, H, W, patch_radius and precision.
 * Errors: INVALID_ARG / UNSUPPORTED as segsalsa_str_solve would return them.
 */
segsalsa_status segsalsa_str_workspace_size(const segsalsa_problem *prob, segsalsa_precision precision,
                                            size_t *bytes /* HOST, out */);

/*
 * Run prob->iters rounds of SALSA for SegSALSA-STR (Sec. 4, eqs. (12)-(14)).
 *
 *   input      [K][H][W] probabilities p(x_i | y_i = k) (eq. (7)) or logits; read only.
 *   z_out      [K][H][W] hidden field after the last round; must not alias input.
 *              With warm_start it must hold the z of the previous call on entry.
 *   workspace  >= segsalsa_str_workspace_size bytes, 256-byte aligned; holds the
 *              solver state (normalised p, scaled multipliers d1..d4) between
 *              warm-started calls.
 *   stats      HOST, may be NULL.  When given, the call waits for `stream` and
 *              fills it.  Required when residual_every > 0 or tol > 0.
 *
 * Invalid probabilities (negative, non-finite, zero-sum pixels) are not
 * detected on the host; the device check sets stats->flags and the result
 * is then undefined.
 */
segsalsa_status segsalsa_str_solve(const segsalsa_problem *prob, segsalsa_precision precision,
                                   const void *input, void *z_out, void *workspace, size_t workspace_bytes,
                                   segsalsa_stats *stats, hipStream_t stream);

/*
 * segsalsa_str_solve for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  It takes no workspace: the solver state lives in a device
 * array of SEGSALSA_NOALLOC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends, and the call allocates nothing
 * (no hipMalloc or hipFree, no graph, no events).  The caller still owns
 * input and z_out, with the meaning of segsalsa_str_solve.
 *  - A problem whose workspace (segsalsa_str_workspace_size) is larger than
 *    the array returns UNSUPPORTED.
 *  - use_graph, residual_every and tol must be 0 (INVALID_ARG); there are no
 *    stats.  The launches are plain kernel launches on `stream` and can be
 *    captured into the caller's own graph.
 *  - Every call on one GPU uses that GPU's single array and leaves its state
 *    there; each call initialises the state it needs (unless warm_start).
 *    Calls that overlap on one GPU (on other streams or threads) race for the
 *    array and give undefined results.  A warm_start call continues from the
 *    state of the previous call on that GPU, which must have had the same
 *    problem and precision.
 */
#define SEGSALSA_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
segsalsa_status segsalsa_str_solve_noalloc(const segsalsa_problem *prob, segsalsa_precision precision,
                                           const void *input, void *z_out, hipStream_t stream);

/* One image of a batch: shape, SALSA parameters, and element offsets of its
 * [K][H][W] input and output inside the packed batch buffers. */
typedef struct {
  int32_t K, H, W;        /* as in segsalsa_problem                                       */
  int64_t in_offset;      /* first element of the image in input_packed (>= 0)             */
  int64_t out_offset;     /* first element of the image in z_packed (>= 0); output ranges
                             must not overlap                                              */
  double lambda, mu;      /* prior weight (>= 0) and SALSA penalty (> 0) of this image     */
} segsalsa_image;

/* Parameters shared by all images of a batch (same meaning as in segsalsa_problem). */
typedef struct {
  int32_t patch_radius;
  const double *patch_weights;   /* HOST, L multipliers c_j                               */
  double schatten_p;
  int32_t iters;
  int32_t input_is_logits;
  int32_t residual_every;        /* with tol > 0 each image stops on its own: an image whose
                                    residuals are <= tol leaves the later launches           */
  double tol;
  int32_t warm_start;
  int32_t use_graph;
  int32_t g4_simplex;
} segsalsa_batch_params;

/* Workspace bytes of segsalsa_str_solve_batch for these images (HOST arrays). */
segsalsa_status segsalsa_str_batch_workspace_size(int32_t n_images, const segsalsa_image *images,
                                                  const segsalsa_batch_params *params,
                                                  segsalsa_precision precision, size_t *bytes /* HOST, out */);

/*
 * SegSALSA-STR on many images of different sizes and class counts at once
 * (the rounds of Sec. 4 on each image).  Every round is one launch per
 * kernel for the whole batch (the proximity kernel: one launch per distinct
 * workgroup shape), so small images share the GPU.
 *
 *   images         HOST, n_images descriptors.
 *   input_packed   device buffer holding every image's input at its in_offset.
 *   z_packed       device buffer receiving every image's z at its out_offset.
 *   stats          HOST, n_images entries or NULL (required with residuals).
 * The result of each image equals segsalsa_str_solve on that image alone to
 * rounding, and bit for bit when both run the same kernels: the batch keeps
 * the planner's tiles and plans its FFT blocking by transform length only (so
 * that images of one length share a launch), which does not change the
 * arithmetic; they differ where the tuning table has an entry for the shape.
 */
segsalsa_status segsalsa_str_solve_batch(int32_t n_images, const segsalsa_image *images,
                                         const segsalsa_batch_params *params, segsalsa_precision precision,
                                         const void *input_packed, void *z_packed, void *workspace,
                                         size_t workspace_bytes, segsalsa_stats *stats, hipStream_t stream);

/*
 * Labels y_i = argmax_k z_ki, lowest k on ties (the segmentation read out of
 * the hidden field, Fig. 1).  z [K][H][W], labels [H][W] int32.
 */
segsalsa_status segsalsa_str_labels(int32_t K, int32_t H, int32_t W, segsalsa_precision precision,
                                    const void *z, int32_t *labels, hipStream_t stream);

/*
 * Copy the solver state held in `workspace` after a solve into canonical
 * layouts: d1, d3, d4 as [K][H][W] and d2 as [L][2][K][H][W] (offset j,
 * direction h/v, class, row, column), the scaled multipliers of the four
 * splits of eq. (11).  Any output pointer may be NULL to skip it.
 */
segsalsa_status segsalsa_str_state_export(const segsalsa_problem *prob, segsalsa_precision precision,
                                          const void *workspace, size_t workspace_bytes, void *d1, void *d2,
                                          void *d3, void *d4, hipStream_t stream);

/*
 * Load a state (normalised probabilities p_hat [K][H][W] and d1..d4 in the
 * layouts of segsalsa_str_state_export) into `workspace`, so that a
 * following warm-started solve continues from it (with z in z_out).
 * All four d pointers and p_hat are required.
 */
segsalsa_status segsalsa_str_state_import(const segsalsa_problem *prob, segsalsa_precision precision,
                                          void *workspace, size_t workspace_bytes, const void *p_hat,
                                          const void *d1, const void *d2, const void *d3, const void *d4,
                                          hipStream_t stream);

/*
 * Differentiable solve: gradients of a loss of the final z with respect to
 * the input, lambda and the patch multipliers c_j, by the reverse sweep of
 * the unrolled rounds of eqs. (12)-(14) (the method's iteration is
 * differentiated as run; the paper itself does not train through it).
 *
 * segsalsa_str_solve_ckpt runs prob->iters rounds like segsalsa_str_solve
 * (same z_out) and keeps, in `workspace`, the state (z, d1..d4) at rounds 0,
 * S, 2S, ... with S = checkpoint_every (clamped to [1, iters]) and the final
 * z.  checkpoint_every = 0 picks S: the smallest interval whose kept states
 * (ceil(iters / S) checkpoints and S - 1 recomputed ones) take at most 8 GiB,
 * else ceil(sqrt(iters)); S = 1 keeps every state and recomputes nothing.
 * The rounds write each state straight into its slot (no copies).
 * segsalsa_str_backward then, given dL/dz_out, recomputes each segment of
 * S rounds from its checkpoint and runs the reverse rounds, and writes
 *   grad_input    [K][H][W]  dL/d input (probabilities or logits, as given);
 *   grad_lambda   DEVICE, 1 double, dL/d lambda (may be NULL);
 *   grad_weights  DEVICE, L doubles, dL/d c_j (may be NULL).
 * The two calls must get the same problem, precision, checkpoint_every,
 * input and workspace, with the workspace untouched in between.  Memory:
 * about (ceil(iters / S) + S) states of (3 + 2L) K H W elements each.
 * The gradient is the derivative of the closed forms that the forward
 * rounds evaluate, taken on the side each branch of the proximity
 * operators computes (max(v, 0) has slope 1 for v > 0 only; the Schatten
 * shrink is differentiated through its eigenvalues, with the divided
 * difference at merged singular values).
 * Restrictions (SEGSALSA_ERR_UNSUPPORTED): residual_every, tol, warm_start,
 * use_graph and g4_simplex must be 0, and schatten_p must be 1, 2 or inf.
 */
segsalsa_status segsalsa_str_grad_workspace_size(const segsalsa_problem *prob, segsalsa_precision precision,
                                                 int32_t checkpoint_every, size_t *bytes /* HOST, out */);
/* The interval S that checkpoint_every (0 = automatic) resolves to for this problem. */
segsalsa_status segsalsa_str_grad_checkpoint_interval(const segsalsa_problem *prob, segsalsa_precision precision,
                                                      int32_t checkpoint_every, int32_t *interval /* HOST, out */);
segsalsa_status segsalsa_str_solve_ckpt(const segsalsa_problem *prob, segsalsa_precision precision,
                                        int32_t checkpoint_every, const void *input, void *z_out, void *workspace,
                                        size_t workspace_bytes, hipStream_t stream);
segsalsa_status segsalsa_str_backward(const segsalsa_problem *prob, segsalsa_precision precision,
                                      int32_t checkpoint_every, const void *input, const void *grad_z,
                                      void *grad_input, double *grad_lambda, double *grad_weights, void *workspace,
                                      size_t workspace_bytes, hipStream_t stream);

/*
 * Launch shapes (not part of the method).  The planner picks, per image
 * shape (K, H, W, patch_radius, precision), the prox kernel's tile and
 * classes per wavefront and the blocking of the FFT passes from a cost
 * model.  A process-wide tuning table, filled by segsalsa_str_autotune
 * (measured on the device) or by the caller, overrides those choices for the
 * shapes it holds in forward solves of one image (segsalsa_str_solve, the
 * graph and no-allocation variants).  The differentiable solve and batches of
 * more than one image keep the planner's shapes: the entries are measured
 * with the image alone on the device, while a batch's images share it and
 * the planner's shapes group them into fewer launches.  A tuned entry
 * changes the launch shapes and the workspace size, not the arithmetic: the
 * results agree with untuned ones to rounding (the fold and the class sums
 * are added in another order).  Size workspaces after changing the table.
 * All functions are thread-safe.
 */
typedef struct {
  int32_t tile_rows, tile_cols;  /* prox tile in pixels (both > 0), or 0 for the planner's            */
  int32_t classes_per_wave;      /* classes per wavefront of the prox kernel: 1, 2 or 4, or 0          */
  int32_t prefetch;              /* 1: the prox kernel build that loads step s + 1 while step s
                                    updates (FP32, classes_per_wave = 2, patch radius <= 2); 0: not    */
  int32_t generic_fft;           /* 1: the general mixed-radix FFT kernels (Bluestein in LDS) also for
                                    the sides that otherwise take the fixed-structure engine: powers of
                                    two 64 .. 4096 (N / 16 threads per transform) and sides taking
                                    Bluestein with a convolution length M of 64 .. 4096 (M / 16 threads
                                    per transform); with the engine, threads are rows or columns per
                                    block times N / 16 or M / 16                                       */
  int32_t col_dft;               /* 1: the column pass by DFTs (column DFT, symbol, inverse DFT); 0: by
                                    the exact periodic tridiagonal recursions per column frequency,
                                    cols_per_block columns of ceil(H / 32) (FP64: ceil(H / 16)) threads
                                    each, col_threads >= their product.  FP32 solves whose weights put
                                    the recursions' largest rho = 2 Wsum / (a + sqrt(a^2 - 4 Wsum^2)),
                                    a = 3 + 2 Wsum, within 0.1 of 1 (Wsum above ~280) take the DFT pass
                                    whatever this field says (the recursions' rounding grows like
                                    eps / (1 - rho)), and then ignore a tuned recursion blocking       */
  int32_t rows_per_block;        /* rows per workgroup of the row DFT passes (> 0), or 0               */
  int32_t row_threads;           /* threads per row workgroup, a multiple of 64 in [64, 1024], or 0    */
  int32_t cols_per_block;        /* columns per workgroup of the column pass (> 0), or 0               */
  int32_t col_threads;           /* threads per column workgroup, as row_threads, or 0                 */
  double us_per_round;           /* measured microseconds per round with this entry (0 = not measured) */
} segsalsa_tuning;

/* Set (or, with tuning == NULL, remove) the entry of one shape.  The entry is
 * checked against the planner's limits (LDS, registers, fold lists) and
 * refused with INVALID_ARG / UNSUPPORTED if it does not fit. */
segsalsa_status segsalsa_tuning_set(int32_t K, int32_t H, int32_t W, int32_t patch_radius,
                                    segsalsa_precision precision, const segsalsa_tuning *tuning /* HOST */);
/* The shapes the planner uses for this image shape (every field filled in) and
 * whether they come from the table (*tuned = 1) or the cost model (0). */
segsalsa_status segsalsa_tuning_get(int32_t K, int32_t H, int32_t W, int32_t patch_radius,
                                    segsalsa_precision precision, segsalsa_tuning *out /* HOST */,
                                    int32_t *tuned /* HOST, may be NULL */);
/* Remove every entry. */
segsalsa_status segsalsa_tuning_clear(void);
/* Read entries from a JSON tuning cache written by segsalsa_tuning_save and
 * add them to the table (entries that do not fit are skipped and counted in
 * *skipped, which may be NULL).  A missing or unreadable file is INVALID_ARG. */
segsalsa_status segsalsa_tuning_load(const char *path, int32_t *loaded /* HOST, may be NULL */,
                                     int32_t *skipped /* HOST, may be NULL */);
/* Write the whole table as a JSON tuning cache. */
segsalsa_status segsalsa_tuning_save(const char *path);

/* The launch shapes each image of this batch runs with (not part of the
 * method): plans[i] (HOST, n_images entries) receives image i's prox tile,
 * classes per wavefront and FFT blocking, as segsalsa_tuning_get reports them
 * for single images (us_per_round = 0). */
segsalsa_status segsalsa_str_batch_plans(int32_t n_images, const segsalsa_image *images,
                                         const segsalsa_batch_params *params, segsalsa_precision precision,
                                         segsalsa_tuning *plans /* HOST, out */);

/*
 * Measure launch shapes for `prob`'s image shape on the device and store the
 * fastest in the tuning table (and in *best if given).  Coordinate search:
 * prox tile and classes per wavefront by the time of whole rounds, then the
 * row DFT blocking by the time of the two row passes, then the column
 * blocking by the time of the column pass; each candidate runs the
 * initialisation from `input` and 1 + rounds rounds (rounds in [1, 100]) and
 * is timed with HIP events on `stream`.  Waits for `stream`.  z_scratch is a
 * [K][H][W] array of the precision's type that receives z (overwritten).
 * The workspace must hold segsalsa_str_autotune_workspace_size bytes (the
 * largest candidate's).  Only prob's shape, patch radius, weights, p,
 * lambda and mu are used (a fixed-round forward solve).
 */
segsalsa_status segsalsa_str_autotune_workspace_size(const segsalsa_problem *prob, segsalsa_precision precision,
                                                     size_t *bytes /* HOST, out */);
segsalsa_status segsalsa_str_autotune(const segsalsa_problem *prob, segsalsa_precision precision,
                                      const void *input, void *z_scratch, void *workspace, size_t workspace_bytes,
                                      int32_t rounds, segsalsa_tuning *best /* HOST, may be NULL */,
                                      hipStream_t stream);

/*
 * Instrumentation (not part of the method): per-phase GPU time of the rounds
 * enqueued by segsalsa_str_solve, measured with HIP events recorded on the
 * caller's stream immediately before and after each kernel launch.  Off by
 * default; enabling it adds two event records per launch.
 *   phases: 0 = fused proximity/multiplier/J^T kernel, 1 = fold + row DFT,
 *           2 = column half of the solve (the recursions, or column DFT /
 *           symbol division / inverse column DFT),
 *           3 = inverse row DFT, 4 = reverse-sweep proximity kernel
 *           (segsalsa_str_backward; its solves count under 1-3).
 * segsalsa_profile_read waits for the recorded events, adds their elapsed
 * times to running per-phase totals, and copies the totals (milliseconds and
 * launch counts, SEGSALSA_NUM_PHASES entries each, HOST, either may be NULL);
 * reset != 0 clears the totals afterwards.  Thread-safe.
 */
#define SEGSALSA_NUM_PHASES 5
segsalsa_status segsalsa_profile_enable(int32_t on);
segsalsa_status segsalsa_profile_read(double *ms, int64_t *launches, int32_t reset);

/*
 * Instrumentation (not part of the method), for callers that measure the
 * memory system's streaming rate as the reference of the proximity kernel's
 * roofline: copies `bytes` from src to dst (both DEVICE, caller-owned,
 * 16-byte aligned, not overlapping; bytes a multiple of 16) with 16-byte
 * nontemporal loads and stores, the access pattern of that kernel's
 * streaming build.  Asynchronous on `stream`; INVALID_ARG for NULL, misaligned
 * or overlapping buffers (checked on the host, nothing is launched).
 */
segsalsa_status segsalsa_stream_copy(const void *src /* DEVICE */, void *dst /* DEVICE */, size_t bytes,
                                     hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SEGSALSA_H */
