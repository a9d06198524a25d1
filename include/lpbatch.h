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
 * reduced costs); a basis that fails that certificate is re-solved from
 * scratch in double precision, so reported results carry FP64 accuracy. */
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
#define LP_STAT_FALLBACK 3      /* 1: the FP64 re-solve (or warm-start fallback) ran */
#define LP_STAT_REFINE 4        /* FP64 pivots of the fallback solve                 */
#define LP_STAT_CERT 5          /* certificate outcome, LP_CERT_* bits              */
#define LP_STAT_PLACEMENT 6     /* where the tableau lived, LP_PLACE_*              */
#define LP_STAT_BASIC_STRUCT 7  /* basic structural variables at the end            */

#define LP_CERT_PRIMAL_OK 1
#define LP_CERT_DUAL_OK 2
#define LP_CERT_RAY_OK 4
#define LP_CERT_SINGULAR 8

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
                            tableau in a device scratch slot, workgroup kernel)   */
    int32_t block_threads; /* 0 auto: LPs of <= 63 columns and <= 128 rows get one
                            wavefront each, others a workgroup; 64, 128, 256 or
                            512: every LP gets a workgroup of that many threads  */
    int32_t *stats;      /* optional DEVICE int32 [num_lps][LP_STATS_WIDTH]       */
    void *stream;        /* hipStream_t the work is queued on; NULL: null stream  */
    uint32_t flags;      /* LP_FLAG_*                                              */
} lp_options;

#define LP_FLAG_SYNC 1u        /* wait for the stream before returning            */
#define LP_FLAG_TIME_KERNELS 2u /* record HIP events around each kernel launched  */

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
 * lp_ctx_kernel_times -- durations of every kernel launched by the context's
 * lp_batch_solve_ex calls made with LP_FLAG_TIME_KERNELS since the previous
 * lp_ctx_kernel_times call, in launch order.  Synchronises on the recorded
 * events, then forgets them.  Writes up to `cap` entries of names[] (static
 * strings) and ms[]; returns how many kernels were recorded, or a negative
 * LP_ERR_* code.
 */
int lp_ctx_kernel_times(lp_ctx *ctx, const char **names, float *ms, int cap);

/* Text of the last failure on the calling thread ("" if none). */
const char *lp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LPBATCH_H */
