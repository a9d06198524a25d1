/*
 * lpbatch.h -- C ABI of the MI355X batched LP solver.
 *
 * Solves many independent linear programs at once with the dense-tableau
 * simplex method (Gurung & Ray, "Simultaneous Solving of Batched Linear
 * Programs on a GPU", arXiv:1802.08557).  Every LP k of a batch is
 *
 *     maximise  c_k^T x   subject to  A_k x  (<=, >=, =)  b_k,   x >= 0
 *
 * -- the standard form of Sec. 4, Eq. (1)-(3), widened to three row senses --
 * and is solved by the two-phase simplex of Sec. 4 / 4.1: Phase I on the
 * auxiliary LP whose objective is the sum of artificial variables when the
 * initial slack basis is infeasible, then Phase II; Step 1 prices the entering
 * column (largest reduced cost, ties to the smallest variable index), Step 2
 * takes the leaving row by the minimum-ratio test (ties to the smallest basic
 * variable index), Step 3 pivots.  After a run of degenerate pivots the
 * entering rule switches to Bland's smallest-index rule until progress resumes.
 *
 * Batch layout.  LPs are stored back to back:
 *   A      double [sum_k m[k]*n[k]]  LP k's m[k] x n[k] block, row-major, at
 *                                    aoff[k] = sum_{t<k} m[t]*n[t]
 *   b      double [sum_k m[k]]       at roff[k] = sum_{t<k} m[t]
 *   sense  int8   [sum_k m[k]]       at roff[k]; values lp_sense
 *   c      double [sum_k n[k]]       at coff[k] = sum_{t<k} n[t]
 *   x      double [sum_k n[k]]       output, at coff[k]
 *   status int32  [num_lps]          output, lp_status
 *   obj    double [num_lps]          output
 * A, b, c, sense, x, status and obj are DEVICE pointers (memory of the GPU the
 * call runs on); m[] and n[] are HOST arrays (the planner reads them before it
 * launches anything).  All memory is owned by the caller; the library never
 * frees or retains a caller pointer after the call's work has completed.
 *
 * Results per LP are statuses, never errors:
 *   LP_OPTIMAL          x is an optimal vertex, obj = c^T x (recomputed in FP64)
 *   LP_INFEASIBLE       obj = NaN, x = NaN
 *   LP_UNBOUNDED        obj = +inf, x = NaN
 *   LP_ITERATION_LIMIT  pivot cap reached; obj = NaN, x = NaN
 *   LP_NUMERICAL        the method broke down (e.g. Phase I unbounded)
 *   LP_INVALID_INPUT    a non-finite entry in A, b or c, or a sense value
 *                       outside 0..2; the rest of the batch still solves
 * Whole-call failures are negative return codes (see LP_ERR_*); the text of
 * the last failure on the calling thread is lp_last_error().
 */
#ifndef LPBATCH_H
#define LPBATCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { LP_LE = 0, LP_GE = 1, LP_EQ = 2 } lp_sense;

typedef enum {
    LP_OPTIMAL = 0,
    LP_INFEASIBLE = 1,
    LP_UNBOUNDED = 2,
    LP_ITERATION_LIMIT = 3,
    LP_NUMERICAL = 4,
    LP_INVALID_INPUT = 5
} lp_status;

/* Arithmetic of the tableau.  LP_PREC_FP64: every pivot in double precision.
 * LP_PREC_FP32_CERT64: pivots on a single-precision tableau, then the final
 * basis is re-solved in double precision on the GPU (x_B = B^-1 b, duals,
 * reduced costs; the ray of an unbounded result; the Phase I duals of an
 * infeasible one, see LP_CERT_*); a result that fails that certificate is
 * refined in double precision from its final basis, or re-solved from the
 * slack basis when that is not possible, so reported results carry FP64
 * accuracy. */
typedef enum { LP_PREC_FP64 = 0, LP_PREC_FP32_CERT64 = 1 } lp_precision;

#define LP_OK 0
#define LP_ERR_ARG (-1)   /* null pointer, num_lps < 0, m or n < 1, size overflow */
#define LP_ERR_NOMEM (-2) /* device scratch could not be allocated                */
#define LP_ERR_HIP (-3)   /* a HIP runtime call failed (text in lp_last_error)    */

/* Width of one LP's row in lp_options.stats. */
#define LP_STATS_WIDTH 8
/* stats[k][LP_STAT_*]: */
#define LP_STAT_PIVOTS_PHASE1 0 /* Phase I pivots                                    */
#define LP_STAT_PIVOTS_PHASE2 1 /* Phase II pivots                                   */
#define LP_STAT_DEGENERATE 2    /* pivots with a zero step                           */
#define LP_STAT_FALLBACK 3      /* 1: the FP64 re-solve ran from the slack basis;
                                   2: it started from the single-precision (or the
                                   screened relaxation's) final basis              */
#define LP_STAT_REFINE 4        /* FP64 pivots of the fallback solve                 */
#define LP_STAT_CERT 5          /* certificate outcome, LP_CERT_* bits              */
#define LP_STAT_PLACEMENT 6     /* where the tableau lived, LP_PLACE_*              */
#define LP_STAT_BASIC_STRUCT 7  /* basic structural variables at the end            */

#define LP_CERT_PRIMAL_OK 1 /* x_B = B^-1 b and every row's slack within tolerance   */
#define LP_CERT_DUAL_OK 2   /* every reduced cost and dual sign within tolerance     */
/* An unbounded result: the FP64 ray of the entering column keeps every basic
 * variable and row feasible and raises the objective, and the LP has a
 * feasible point (the basis passes the primal check, or x = 0 is feasible). */
#define LP_CERT_RAY_OK 4
#define LP_CERT_SINGULAR 8  /* the basis block could not be factorised          */
/* An infeasible result proven in FP64 from the FP32 solve's final Phase I
 * basis (Phase I optimum below zero, every structural and slack reduced cost
 * within tolerance: -y is a Farkas certificate).  Given by the workgroup
 * certificate (LPs with their own constraints and more than 64 rows and
 * columns); other infeasible results are re-solved in FP64. */
#define LP_CERT_INFEASIBLE_OK 16

#define LP_PLACE_LDS 1    /* tableau in LDS (stats: one wavefront per LP)    */
#define LP_PLACE_HBM 2    /* tableau in a device-memory slot (workgroup)     */
#define LP_PLACE_LDS_WG 3 /* stats only: tableau in LDS, one workgroup per LP */

/*
 * lp_batch_solve -- solve a batch in FP64 on the current device, synchronously.
 *
 * Uses a library-owned context for the current device (created on first use)
 * and the null stream; returns after every result has been written.
 * Returns LP_OK or a negative LP_ERR_* code; per-LP outcomes go to status[].
 */
int lp_batch_solve(int64_t num_lps, const double *A, const double *b, const double *c,
                   const int8_t *sense, const int32_t *m, const int32_t *n,
                   int32_t *status, double *x, double *obj);

/* A solver context: device scratch (grow-only), the tuned placement table,
 * launch plans and timing events for one device.  Not thread-safe: one
 * context per host thread, or external locking. */
typedef struct lp_ctx lp_ctx;

/* Creates a context on `device` (a HIP device ordinal).  Returns LP_OK or
 * LP_ERR_ARG / LP_ERR_HIP. */
int lp_ctx_create(lp_ctx **out, int device);
void lp_ctx_destroy(lp_ctx *ctx);

/* Options of lp_batch_solve_ex.  Zero-initialised fields mean "default";
 * lp_options_init fills the defaults explicitly. */
typedef struct {
    int32_t precision;   /* lp_precision                                          */
    int32_t max_iters;   /* pivot cap over both phases; 0: 50 * (m + #columns)   */
    double tol_piv;      /* pivot-entry threshold; 0: 1e-9 (FP64), 1e-6 (FP32)    */
    double tol_opt;      /* reduced-cost threshold, relative to max(1, |c|_inf)   */
    double tol_feas;     /* Phase I optimum threshold, relative to 1 + |b|_inf   */
    int32_t k_deg;       /* degenerate pivots before Bland's rule; 0: 50; <0: off */
    int32_t placement;   /* 0 auto, LP_PLACE_LDS or LP_PLACE_HBM (HBM: every LP's
                            tableau in a device scratch slot, workgroup kernel).
                            Auto keeps a workgroup-kernel tableau in LDS when it
                            takes at most a third of a CU's LDS; LP_PLACE_LDS
                            whenever it fits                                       */
    int32_t block_threads; /* 0 auto: LPs of <= 64 columns and <= 128 rows get one
                            wavefront each, others a workgroup; 64, 128, 256 or
                            512: every LP gets a workgroup of that many threads  */
    int32_t *stats;      /* optional DEVICE int32 [num_lps][LP_STATS_WIDTH]       */
    void *stream;        /* hipStream_t the work is queued on; NULL: null stream  */
    uint32_t flags;      /* LP_FLAG_*                                              */
    /* Shared constraints (the support-function workload of the paper's
     * "Motivating Application" section: one polytope, many objectives).
     * shared = 1: A, b and sense hold ONE LP of m[0] x n[0] that every LP of
     * the batch uses; c, x, status and obj stay per LP; every m[k] must equal
     * m[0] and every n[k] n[0].                                                 */
    int32_t shared;
    /* Screened solve (needs shared = 1): a DEVICE int32 [num_lps][subset_m]
     * list of constraint indices.  LP k is first solved on those rows only --
     * a relaxation, since dropping constraints only enlarges the feasible
     * set -- in the chosen precision.  Its final basis, completed with the
     * slacks of the omitted rows, is then certified in FP64 against EVERY
     * row (primal feasibility of all m rows, reduced costs); an LP whose
     * relaxation is not optimal or whose basis fails is re-solved on all rows
     * in FP64: first from the relaxation's final basis -- its basic
     * structurals pivoted in, then dual simplex pivots restore feasibility on
     * the rows it violates (stats[LP_STAT_FALLBACK] = 2); an LP this repair
     * does not finish optimal (it needs <= rows throughout) is solved from the
     * slack basis (stats[LP_STAT_FALLBACK] = 1).  Results
     * always refer to the full LP.  An index outside 0..m[0]-1 makes that LP
     * LP_INVALID_INPUT in the first pass and sends it to the re-solve.       */
    const int32_t *row_subset;
    int32_t subset_m;    /* rows per LP in row_subset, 1..m[0]                    */
    /* Preconditioning (not part of the paper's method, which pivots on the LP
     * as given, Sec. 4): scaling = P > 0 runs P passes of geometric-mean
     * scaling with power-of-two factors (lp_batch_scale) on a copy of the
     * batch in context scratch, solves the scaled LPs with every other option
     * unchanged (tolerances then apply to the scaled data) and maps x back;
     * status and obj refer to the LP as given.  0: off; at most 64.           */
    int32_t scaling;
    /* Step 1's rule (lp_pricing).  LP_PRICE_DANTZIG: the largest reduced cost
     * d_j, the paper's rule.  LP_PRICE_STEEPEST_EDGE (not in the paper): the
     * largest d_j^2 / (1 + sum_i t_ij^2) over the live rows of the current
     * tableau -- the gain per unit length of the edge column j opens, computed
     * exactly from the tableau at every pricing.  Both hand over to Bland's
     * rule after k_deg degenerate pivots.                                     */
    int32_t pricing;
} lp_options;

typedef enum { LP_PRICE_DANTZIG = 0, LP_PRICE_STEEPEST_EDGE = 1 } lp_pricing;

#define LP_FLAG_SYNC 1u        /* wait for the stream before returning            */
#define LP_FLAG_TIME_KERNELS 2u /* record HIP events around each kernel launched  */
/* Workgroup-kernel launches (paper Sec. 5.1, load balancing): in a batch of
 * mixed LP sizes every LP the one-wavefront kernel cannot take goes to ONE
 * persistent launch of the workgroup kernel whose queue hands out the most
 * expensive LPs first (m n (m + n)), each LP's tableau in LDS when it fits the
 * launch's budget and in the workgroup's device-memory slot otherwise.  The
 * planned shapes stay on the device: a later call on the same context with
 * the same m[] and n[] uploads nothing and does not wait on the host, so it
 * can be captured in a HIP graph (capturing the first solve of a new set of
 * shapes fails with LP_ERR_ARG).  A batch of one size that the workgroup
 * kernel takes is one launch as well.  With LP_FLAG_AUTOTUNE, a launch whose
 * bin is not yet in the context's table -- size bins 0..3 by tableau cells
 * ((m+1)(n+1) <= 64^2, 128^2, 256^2, larger) for batches of one size, bin 4
 * for the launch of a mixed batch -- is first timed on a sample of up to 512
 * of its LPs for each workgroup size (64, 128, 256, 512) and placement (LDS
 * when it fits, or device memory), and the fastest is kept in the context for
 * later calls.  The call is then synchronous; results are as without the
 * flag. */
#define LP_FLAG_AUTOTUNE 4u

void lp_options_init(lp_options *opts);

/*
 * lp_batch_solve_ex -- asynchronous batch solve on opts->stream.
 *
 * Same batch layout and result conventions as lp_batch_solve.  The work is
 * queued on opts->stream and the call returns without waiting unless
 * LP_FLAG_SYNC is set; the caller keeps every buffer alive until that stream
 * has reached the call's work.  opts may be NULL (defaults, null stream).
 * Returns LP_OK or a negative LP_ERR_* code (nothing is queued on failure).
 */
int lp_batch_solve_ex(lp_ctx *ctx, int64_t num_lps, const double *A, const double *b,
                      const double *c, const int8_t *sense, const int32_t *m,
                      const int32_t *n, int32_t *status, double *x, double *obj,
                      const lp_options *opts);

/*
 * lp_batch_solve_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the solve of lp_batch_solve_ex with default options in FP64 for
 * a batch of ONE shape (every LP m x n, so m and n are scalars here) that the
 * one-wavefront kernel takes -- n <= 64, m <= 128, the m x n FP64 tableau in a
 * CU's LDS -- with the same kernels and bit-for-bit the same results.
 *
 * A, b, c, sense, status, x, obj: DEVICE pointers, laid out as for
 * lp_batch_solve_ex (uniform shape: LP k's A at k*m*n, b and sense at k*m, c and
 * x at k*n); stats: optional DEVICE int32 [num_lps][LP_STATS_WIDTH] or NULL.
 * The work is queued on `stream` (hipStream_t; NULL: null stream) and the call
 * returns without waiting; the caller keeps the buffers alive until then.
 *
 * The call allocates nothing: its work counters, the list of LPs the
 * wavefront kernel defers (rows >= after normalisation add surplus columns
 * past 64) and the workgroup-kernel tableau slots that solve those live in a
 * statically allocated 16 MiB device array that each device holds from the
 * moment the library is loaded there until the process ends.  Limits:
 * num_lps <= 2^20 (LP_ERR_ARG beyond); the shape limits above (LP_ERR_ARG).
 * Every call on a device shares that device's array and the array keeps the
 * last call's contents (the call clears what must start at zero): calls that
 * overlap on one device -- on different streams or host threads, or through
 * different contexts -- race and must not be issued.  Returns LP_OK or a
 * negative LP_ERR_* code (LP_ERR_HIP also when the array's device address
 * could not be looked up at lp_ctx_create).
 */
int lp_batch_solve_noalloc(lp_ctx *ctx, int64_t num_lps, const double *A, const double *b,
                           const double *c, const int8_t *sense, int32_t m, int32_t n,
                           int32_t *status, double *x, double *obj, int32_t *stats,
                           void *stream);

/*
 * lp_batch_solve_host -- a batch held in HOST memory, streamed through the
 * device in chunks (paper Sec. 5.1, Algorithm 1: the batch is cut into chunks
 * that fit the device, each copied over, solved and copied back; and the
 * transfer overlap of its "Data transfer and kernel execution" discussion).
 *
 * Same batch layout, options and results as lp_batch_solve_ex, except that
 * A, b, c, sense, status, x and obj are HOST pointers (m and n are host arrays
 * as always).  Chunk i's inputs go host -> device on one copy stream, its
 * solve runs on a compute stream once they have arrived, and its status, x
 * and obj go device -> host on a second copy stream; three chunk buffers in
 * rotation let chunk i+1's upload and chunk i-1's download proceed while chunk
 * i is solved.  Host buffers allocated pinned (hipHostMalloc, or a PyTorch
 * tensor with pin_memory) are copied directly; pageable buffers are staged
 * through pinned buffers of the context by the calling thread, which then
 * bounds the rate.
 *
 * chunk_lps: LPs per chunk; 0 chooses min(Eq. (5)-style capacity of a quarter
 * of the free device memory split over three chunk buffers,
 * max(4096, ceil(num_lps / 8))).  opts may be NULL; opts->stats, opts->shared
 * and opts->row_subset must be unset (LP_ERR_ARG otherwise), opts->stream and
 * LP_FLAG_SYNC are ignored: the call is synchronous and returns when every
 * result is in the caller's arrays.  Returns LP_OK or a negative LP_ERR_*
 * code.
 */
int lp_batch_solve_host(lp_ctx *ctx, int64_t num_lps, const double *A, const double *b,
                        const double *c, const int8_t *sense, const int32_t *m,
                        const int32_t *n, int32_t *status, double *x, double *obj,
                        const lp_options *opts, int64_t chunk_lps);

/*
 * lp_ctx_kernel_times -- durations of every kernel launched by the context's
 * lp_batch_solve_ex calls made with LP_FLAG_TIME_KERNELS since the previous
 * lp_ctx_kernel_times call, in launch order.  Synchronises on the recorded
 * events, then forgets them.  Writes up to `cap` entries of names[] (static
 * strings) and ms[]; returns how many kernels were recorded, or a negative
 * LP_ERR_* code.
 */
int lp_ctx_kernel_times(lp_ctx *ctx, const char **names, float *ms, int cap);

/*
 * lp_ctx_tuning -- the context's autotuned launches, up to `cap` entries of
 * 4 int32 each (HOST memory): bin (0..3: size bin of a batch of one size; 4:
 * the launch of a mixed batch), 1 for FP32 tableaux, workgroup size, 1 when
 * tableaux go to device memory.  Returns the number of entries
 * the table holds (entries may be NULL to count), or a negative LP_ERR_* code.
 */
int lp_ctx_tuning(lp_ctx *ctx, int32_t *entries, int cap);

/*
 * lp_batch_scale -- geometric-mean scaling with power-of-two factors, the
 * preconditioning behind lp_options.scaling (the paper applies none: its
 * tableau is built from the LP as given, Sec. 4).
 *
 * For LP k (layout as in lp_batch_solve) let E_ij = floor(log2 |a_ij|) over
 * the finite non-zero entries.  Starting from s_j = 0, each of `passes`
 * passes sets, for every row with such entries,
 *     r_i = -floor((max_j (E_ij + s_j) + min_j (E_ij + s_j) + 1) / 2),
 * then s_j the same way down every column with the new r_i; rows and columns
 * without entries get 0, every exponent is clamped to [-128, 128].  Outputs:
 *     A_out[ij] = a_ij 2^(r_i + s_j),  b_out[i] = b_i 2^r_i,  c_out[j] = c_j 2^s_j,
 *     row_exp[i] = r_i,  col_exp[j] = s_j,
 * which is the same LP in x'_j = x_j / 2^s_j (exact: powers of two round
 * nothing unless a value leaves the double range).
 * A, b, c, A_out, b_out, c_out, row_exp, col_exp: DEVICE pointers, same
 * layout as the inputs (row_exp [sum m_k], col_exp [sum n_k]); with
 * shared = 1 (every m[k], n[k] equal) A and b hold one LP, c is [num][n[0]],
 * and the exponents are those of the one A ([m[0]], [n[0]]).  m, n: HOST
 * int32 [num_lps].  passes: 0..64 (0 copies with zero exponents).  Outputs
 * must not overlap the inputs.  Queued on stream (NULL: null stream); uneven
 * batches wait for a small upload of their shapes first.  Returns LP_OK or
 * LP_ERR_ARG / LP_ERR_NOMEM / LP_ERR_HIP.
 */
int lp_batch_scale(lp_ctx *ctx, int64_t num_lps, const double *A, const double *b, const double *c,
                   const int32_t *m, const int32_t *n, int32_t passes, int32_t shared, double *A_out,
                   double *b_out, double *c_out, int32_t *row_exp, int32_t *col_exp, void *stream);

/*
 * lp_hyperbox_support -- LPs whose feasible set is a hyper-rectangle, in
 * closed form (paper, "Solving a Special Case of LP", Eq. (7)):
 *
 *   value[k] = max { l_k . x : lo_k <= x <= hi_k } = sum_i l_ki h_ki,
 *   h_ki = lo_ki if l_ki < 0, else hi_ki   (l_ki = 0 takes hi_ki),
 *
 * summed in index order.  l is [num][n]; lo and hi are [num][n], or [n] for
 * one box shared by every direction when shared_box = 1; value is [num]; x
 * (optional, NULL to skip) receives the maximiser h, [num][n].  All DEVICE
 * pointers, row-major; lo <= hi is the caller's to ensure.  Queued on stream
 * (NULL: null stream).  Returns LP_OK or a negative LP_ERR_* code.
 */
int lp_hyperbox_support(lp_ctx *ctx, int64_t num, int32_t n, const double *lo, const double *hi,
                        const double *l, int32_t shared_box, double *value, double *x, void *stream);

/*
 * Warm-start scoring network.
 *
 * For many LPs that share one constraint set and differ only in the objective
 * -- the support-function queries max l^T x over a fixed polytope that the
 * paper's "Motivating Application" section solves in bulk -- a small network
 * maps the direction l to one score per constraint; high scores mark the
 * constraints expected to be tight at the optimum.  The scores choose the rows
 * of the relaxed LP that lp_options.row_subset solves first.  The paper has no
 * learned component; this is an addition around its method.
 *
 * Architecture 20 -> 256 -> 256 -> 120 with ReLU.  Parameters are one FP32
 * vector of LP_MLP_NUM_PARAMS values in the order W1 [256][20], b1 [256],
 * W2 [256][256], b2 [256], W3 [120][256], b3 [120] (row-major, output index
 * first).  Matrix products take BF16 operands (weights, inputs and hidden
 * activations rounded to nearest-even) and accumulate in FP32 on the matrix
 * cores; biases, scores and gradients are FP32.  Training minimises the mean
 * binary cross-entropy with logits over all B x 120 outputs with AdamW
 * (beta1 0.9, beta2 0.999, eps 1e-8, decoupled weight decay on W1, W2, W3).
 *
 * The network lives in the context.  Every pointer argument except `path` is
 * a DEVICE pointer; work is queued on `stream` (NULL: null stream) and the
 * context's buffers are reused by the next call, so calls on one context must
 * be ordered on one stream.  Returns LP_OK or a negative LP_ERR_* code.
 */
#define LP_MLP_IN 20
#define LP_MLP_HIDDEN 256
#define LP_MLP_OUT 120
#define LP_MLP_NUM_PARAMS 102008

/* Fresh parameters: weights uniform in +-sqrt(6 / fan_in) from a splitmix64
 * stream seeded by `seed`, zero biases; clears the AdamW state.  Synchronous. */
int lp_mlp_init(lp_ctx *ctx, uint64_t seed);
/* Copies LP_MLP_NUM_PARAMS FP32 parameters in (clears the AdamW state) or out. */
int lp_mlp_set_params(lp_ctx *ctx, const float *params, void *stream);
int lp_mlp_get_params(lp_ctx *ctx, float *params, void *stream);
/* Scores of B directions dirs [B][20] (FP32): scores [B][120] (optional) and
 * top_k [B][k] (optional, 1 <= k <= 120): the indices of the k highest scores
 * of each row, highest first, equal scores lower index first. */
int lp_mlp_infer(lp_ctx *ctx, int64_t B, const float *dirs, float *scores, int32_t *top_k,
                 int32_t k, void *stream);
/* Gradient of the loss on B labelled rows (tight [B][120]: 1 = tight) into
 * grad_out [LP_MLP_NUM_PARAMS] and the loss into loss_out[0] (either optional);
 * the parameters are not changed. */
int lp_mlp_grads(lp_ctx *ctx, int64_t B, const float *dirs, const uint8_t *tight,
                 float *grad_out, float *loss_out, void *stream);
/* One AdamW step on B labelled rows; the loss before the step goes to
 * loss_out[0] (optional). */
int lp_mlp_train_step(lp_ctx *ctx, int64_t B, const float *dirs, const uint8_t *tight,
                      float lr, float weight_decay, float *loss_out, void *stream);
/* Parameters and AdamW state to / from a file (host path); synchronous. */
int lp_mlp_save(lp_ctx *ctx, const char *path);
int lp_mlp_load(lp_ctx *ctx, const char *path);

/*
 * lp_measure_peaks -- measured bandwidth of the memory tiers the solve kernels
 * are priced against.  A pivot (paper Sec. 4.1, Step 3, and its
 * implementation discussion around Listing 1) is a rank-1 update -- one fma
 * per tableau element against one read and one write of it -- so a solve is
 * bound by the bandwidth of wherever its tableau lives: LDS for tableaux
 * resident on a CU, device memory (HBM) for streamed ones.  Each figure is the
 * best of three timed launches on the context's device, in bytes per second:
 *   lds_read        16-byte reads, each wavefront reading 1 KB of consecutive
 *                   LDS addresses per instruction (bank-conflict free);
 *   lds_write       the same pattern written;
 *   lds_read_write  each 16-byte slot read and then written back, bytes read
 *                   plus bytes written (the pattern of the pivot's row sweep);
 *   lds_broadcast   bytes delivered to lanes when every lane of a wavefront
 *                   reads the same 16 bytes (the pivot column's values);
 *   hbm_copy        bytes read plus bytes written by a 16-byte-vector copy of
 *                   1 GiB in device memory;
 * clock_hz is the shader clock during the LDS read run (its clock counter
 * against the constant 100 MHz reference counter), num_cu the CU count.  The
 * LDS runs use sixteen wavefronts per CU.  Synchronous; allocates and frees
 * about 2 GiB of device memory.  Returns LP_OK, LP_ERR_ARG (NULL argument) or
 * LP_ERR_HIP.
 */
typedef struct {
    double lds_read, lds_write, lds_read_write, lds_broadcast, hbm_copy;
    double clock_hz;
    int32_t num_cu;
} lp_peaks;

int lp_measure_peaks(lp_ctx *ctx, lp_peaks *out);

/* Text of the last failure on the calling thread ("" if none). */
const char *lp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LPBATCH_H */
