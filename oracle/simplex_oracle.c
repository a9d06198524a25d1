/*
 * simplex_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of the dense-tableau
 * two-phase simplex method of Gurung & Ray, "Simultaneous Solving of Batched
 * Linear Programs on a GPU" (arXiv:1802.08557), in double precision.  It exists
 * to check the GPU library; nothing in the product path may call it.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * What it computes, for every LP of a batch:
 *     maximise  c^T x   subject to  a_i^T x  (<=, >=, =)  b_i,   x >= 0
 * (the standard form of Sec. 4, Eq. (1)-(3), widened to all three senses),
 * returning status OPTIMAL / INFEASIBLE / UNBOUNDED / ITERATION_LIMIT, the
 * optimal objective and a maximiser x.
 *
 * How (paper Sec. 4 and 4.1; every reading of a silent or ambiguous passage is
 * listed in the design doc and repeated at the spot where it is used):
 *   1. Rows with b_i < 0 are negated and their sense flipped, so the right-hand
 *      side is non-negative (Sec. 4: a negative b_i makes the initial basic
 *      solution infeasible).
 *   2. Slack form (Eq. 4): a slack (+1) column for every <= row, a surplus (-1)
 *      column for every >= row, and an artificial (+1) column for every >= and
 *      = row.  Column order = Bland order: structurals 0..n-1, then the
 *      slack/surplus columns in row order, then the artificials in row order.
 *   3. The full simplex tableau of Sec. 4.1: m constraint rows plus the
 *      objective row last, every variable column plus the right-hand side.
 *      The objective row holds the reduced costs d_j (a column may enter when
 *      d_j > 0) and, in the right-hand-side cell, minus the current objective.
 *   4. Phase I (Sec. 4): if any artificial exists, maximise w = -(sum of the
 *      artificials), priced out over the initial basis.  A negative optimum
 *      means INFEASIBLE.  Artificials still basic at zero are driven out by a
 *      pivot on the smallest-index non-artificial column with a non-zero
 *      entry; a row with no such entry is redundant and dropped.  Artificial
 *      columns are dropped (an artificial that leaves the basis never returns).
 *   5. Phase II: the objective row is reset to c and priced out over the
 *      current basis (the "appropriate substitutions" of Sec. 4).
 *   6. The simplex loop of Sec. 4.1:
 *        Step 1, entering column: the largest d_j > eps_opt (Dantzig's rule,
 *          the "most common rule"), ties to the smallest column index.  After
 *          K_deg consecutive degenerate pivots the smallest eligible index is
 *          taken instead (Bland's rule) until a pivot makes progress.
 *        Step 2, leaving row: among rows with a_ie > eps_piv, the minimum
 *          ratio max(b_i, 0) / a_ie, exact ties to the row whose basic
 *          variable has the smallest index.  No such row: UNBOUNDED.
 *        Step 3, pivot: the pivot row is divided by the pivot element, every
 *          other row (objective row included) has a_ie times the new pivot row
 *          subtracted (the update of Listing 1), and the entering column is
 *          set to the exact unit vector.
 *      No entering column: OPTIMAL.  An iteration cap gives ITERATION_LIMIT.
 *   7. x_j = b_i for the row whose basic variable is j, else 0; the objective
 *      is recomputed as sum_j c_j x_j from the input c.
 *
 * Floating-point contraction is disabled when this file is built, so every
 * operation is a single IEEE double rounding, as written.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OPTIMAL = 0, OR_INFEASIBLE = 1, OR_UNBOUNDED = 2, OR_ITERATION_LIMIT = 3,
       OR_NUMERICAL = 4, OR_INVALID_INPUT = 5 };
enum { OR_LE = 0, OR_GE = 1, OR_EQ = 2 };

typedef struct {
    double tol_piv;   /* eligibility of a pivot-column entry in the ratio test  */
    double tol_opt;   /* relative optimality tolerance on reduced costs         */
    double tol_feas;  /* relative tolerance on the Phase I optimum              */
    int32_t k_deg;    /* consecutive degenerate pivots before Bland's rule; <=0: never */
    int32_t max_iters;/* pivot cap over both phases; <= 0: 50 * (m + #columns)  */
    int32_t pricing;  /* 0: Dantzig (the paper's Step 1); 1: steepest edge      */
} oracle_params;

typedef struct {
    double *buf;         /* snapshots of the whole tableau, (m+1) x (ncol+1) each */
    int cap, count;
} trace_rec;

typedef struct {
    int m, n, ncol;      /* rows, structurals, variable columns (no rhs)       */
    int ld;              /* ncol + 1: row length including the rhs column      */
    double *t;           /* (m + 1) x ld, objective row last                    */
    int *basis;          /* basic column of each row                            */
    char *is_basic;      /* per column                                          */
    char *is_art;        /* per column: artificial                              */
    char *col_dead;      /* per column: dropped (artificial after Phase I)      */
    char *row_dead;      /* per row: dropped as redundant                       */
    int *bland;          /* Bland index of each column (n+i slack, n+m+i art)   */
    trace_rec *trace;    /* optional tableau snapshots (tiny LPs, for tests)    */
} tableau;

static void snapshot(tableau *tb)
{
    trace_rec *tr = tb->trace;
    if (!tr || tr->count >= tr->cap)
        return;
    const size_t sz = (size_t)(tb->m + 1) * tb->ld;
    memcpy(tr->buf + sz * tr->count, tb->t, sz * sizeof(double));
    ++tr->count;
}

#define T_(tb, i, j) ((tb)->t[(size_t)(i) * (tb)->ld + (j)])

/* Step 3 of Sec. 4.1: the pivot of Listing 1 on a full tableau. */
static void pivot(tableau *tb, int l, int e)
{
    const int ld = tb->ld;
    double *rowl = &T_(tb, l, 0);
    const double pe = rowl[e];
    for (int j = 0; j < ld; ++j)
        rowl[j] = rowl[j] / pe;
    for (int i = 0; i <= tb->m; ++i) {
        if (i == l || (i < tb->m && tb->row_dead[i]))
            continue;
        double *row = &T_(tb, i, 0);
        const double f = row[e];
        if (f == 0.0)
            continue;
        for (int j = 0; j < ld; ++j)
            row[j] = row[j] - f * rowl[j];
    }
    for (int i = 0; i <= tb->m; ++i)
        if (!(i < tb->m && tb->row_dead[i]))
            T_(tb, i, e) = (i == l) ? 1.0 : 0.0;
    tb->is_basic[tb->basis[l]] = 0;
    tb->basis[l] = e;
    tb->is_basic[e] = 1;
    snapshot(tb);
}

/* Objective row <- cost, then priced out over the current basis:
 * d_j = cost_j - sum_i cost_{B(i)} abar_ij, and the rhs cell = -sum_i cost_{B(i)} bbar_i. */
static void price_out(tableau *tb, const double *cost)
{
    double *obj = &T_(tb, tb->m, 0);
    for (int j = 0; j < tb->ncol; ++j)
        obj[j] = cost[j];
    obj[tb->ncol] = 0.0;
    for (int i = 0; i < tb->m; ++i) {
        if (tb->row_dead[i])
            continue;
        const double cb = cost[tb->basis[i]];
        if (cb == 0.0)
            continue;
        const double *row = &T_(tb, i, 0);
        for (int j = 0; j < tb->ld; ++j)
            obj[j] = obj[j] - cb * row[j];
    }
    for (int i = 0; i < tb->m; ++i)
        if (!tb->row_dead[i])
            obj[tb->basis[i]] = 0.0;
    snapshot(tb);
}

/* Steps 1-3 of Sec. 4.1 iterated until a halt condition.
 * Returns OR_OPTIMAL, OR_UNBOUNDED or OR_ITERATION_LIMIT. */
static int simplex_loop(tableau *tb, double eps_opt, const oracle_params *p,
                        int cap, int *iters, int *deg_pivots)
{
    const int rhs = tb->ncol;
    const double *obj = &T_(tb, tb->m, 0);
    int degenerate_run = 0;
    for (;;) {
        if (*iters >= cap)
            return OR_ITERATION_LIMIT;
        const int bland_mode = (p->k_deg > 0 && degenerate_run >= p->k_deg);
        /* Step 1: entering column.  Dantzig: the largest d_j.  Steepest edge
         * (optional, not the paper's rule): the largest d_j^2 / (1 + sum_i t_ij^2)
         * over the live constraint rows -- the squared rate of objective gain
         * per unit length of the edge that column j opens. */
        int e = -1;
        double best = 0.0;
        for (int j = 0; j < tb->ncol; ++j) {
            if (tb->is_basic[j] || tb->col_dead[j] || tb->is_art[j])
                continue;
            const double d = obj[j];
            if (!(d > eps_opt))
                continue;
            if (bland_mode) { e = j; break; }           /* columns are in Bland order */
            double score = d;
            if (p->pricing == 1) {
                double w = 1.0;
                for (int i = 0; i < tb->m; ++i)
                    if (!tb->row_dead[i]) w += T_(tb, i, j) * T_(tb, i, j);
                score = d * d / w;
            }
            if (e < 0 || score > best) { e = j; best = score; } /* strict: ties keep the smaller index */
        }
        if (e < 0)
            return OR_OPTIMAL;
        /* Step 2: leaving row, minimum ratio max(b_i,0)/a_ie over a_ie > eps_piv. */
        int l = -1;
        double best_th = 0.0;
        for (int i = 0; i < tb->m; ++i) {
            if (tb->row_dead[i])
                continue;
            const double a = T_(tb, i, e);
            if (!(a > p->tol_piv))
                continue;
            const double bi = T_(tb, i, rhs);
            const double th = (bi > 0.0 ? bi : 0.0) / a;
            if (l < 0 || th < best_th ||
                (th == best_th && tb->bland[tb->basis[i]] < tb->bland[tb->basis[l]])) {
                l = i;
                best_th = th;
            }
        }
        if (l < 0)
            return OR_UNBOUNDED;
        if (best_th == 0.0) { ++degenerate_run; ++*deg_pivots; }
        else degenerate_run = 0;
        /* Step 3. */
        pivot(tb, l, e);
        ++*iters;
    }
}

static int allfinite(const double *v, size_t k)
{
    for (size_t i = 0; i < k; ++i)
        if (!isfinite(v[i]))
            return 0;
    return 1;
}

/* Solve one LP.  basis_out (m entries, optional) receives the Bland index of the
 * final basic variable of every row (-1 for a dropped redundant row); stats
 * (optional) receives {Phase I pivots, Phase II pivots, degenerate pivots}. */
static int solve_impl(int m, int n, const double *A, const double *b, const double *c,
                      const int8_t *sense, const oracle_params *p,
                      double *x, double *obj_out, int32_t *basis_out, int32_t *stats,
                      trace_rec *trace, int *ncol_out)
{
    int status = OR_OPTIMAL;
    for (int j = 0; j < n; ++j)
        x[j] = NAN;
    *obj_out = NAN;
    if (basis_out)
        for (int i = 0; i < m; ++i)
            basis_out[i] = -1;
    if (stats)
        stats[0] = stats[1] = stats[2] = 0;
    if (m < 1 || n < 1)
        return OR_INVALID_INPUT;
    if (!allfinite(A, (size_t)m * n) || !allfinite(b, (size_t)m) || !allfinite(c, (size_t)n))
        return OR_INVALID_INPUT;
    for (int i = 0; i < m; ++i)
        if (sense[i] < OR_LE || sense[i] > OR_EQ)
            return OR_INVALID_INPUT;

    /* 1. Normalise: make every rhs non-negative. */
    double *sgn = malloc(sizeof(double) * m);
    int *sen = malloc(sizeof(int) * m);
    double bnorm = 0.0, cnorm = 0.0;
    for (int i = 0; i < m; ++i) {
        sgn[i] = (b[i] < 0.0) ? -1.0 : 1.0;
        sen[i] = sense[i];
        if (b[i] < 0.0 && sen[i] != OR_EQ)
            sen[i] = (sen[i] == OR_LE) ? OR_GE : OR_LE;
        if (fabs(b[i]) > bnorm) bnorm = fabs(b[i]);
    }
    for (int j = 0; j < n; ++j)
        if (fabs(c[j]) > cnorm) cnorm = fabs(c[j]);

    /* 2. Columns in Bland order. */
    int nlog = 0, nart = 0;
    for (int i = 0; i < m; ++i) {
        if (sen[i] != OR_EQ) ++nlog;
        if (sen[i] != OR_LE) ++nart;
    }
    tableau tb;
    tb.m = m; tb.n = n; tb.ncol = n + nlog + nart; tb.ld = tb.ncol + 1;
    tb.t = calloc((size_t)(m + 1) * tb.ld, sizeof(double));
    tb.basis = malloc(sizeof(int) * m);
    tb.is_basic = calloc(tb.ncol, 1);
    tb.is_art = calloc(tb.ncol, 1);
    tb.col_dead = calloc(tb.ncol, 1);
    tb.row_dead = calloc(m, 1);
    tb.bland = malloc(sizeof(int) * tb.ncol);
    tb.trace = trace;
    if (ncol_out)
        *ncol_out = tb.ncol;
    for (int j = 0; j < n; ++j)
        tb.bland[j] = j;

    /* 3. Fill the tableau: rows a_i^T x (+ slack | - surplus) (+ artificial) = b_i. */
    int klog = n, kart = n + nlog;
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j)
            T_(&tb, i, j) = sgn[i] * A[(size_t)i * n + j];
        T_(&tb, i, tb.ncol) = sgn[i] * b[i];
        int logical_col = -1, art_col = -1;
        if (sen[i] != OR_EQ) {
            logical_col = klog++;
            T_(&tb, i, logical_col) = (sen[i] == OR_LE) ? 1.0 : -1.0;
            tb.bland[logical_col] = n + i;
        }
        if (sen[i] != OR_LE) {
            art_col = kart++;
            T_(&tb, i, art_col) = 1.0;
            tb.bland[art_col] = n + m + i;
            tb.is_art[art_col] = 1;
        }
        tb.basis[i] = (sen[i] == OR_LE) ? logical_col : art_col;
        tb.is_basic[tb.basis[i]] = 1;
    }

    const int cap = (p->max_iters > 0) ? p->max_iters : 50 * (m + tb.ncol);
    int iters = 0, degp = 0, it1 = 0;
    double *cost = calloc(tb.ncol, sizeof(double));

    /* 4. Phase I. */
    if (nart > 0) {
        for (int j = 0; j < tb.ncol; ++j)
            cost[j] = tb.is_art[j] ? -1.0 : 0.0;
        price_out(&tb, cost);
        double dscale = 1.0;
        for (int j = 0; j < tb.ncol; ++j)
            if (!tb.is_art[j] && fabs(T_(&tb, m, j)) > dscale)
                dscale = fabs(T_(&tb, m, j));
        int r = simplex_loop(&tb, p->tol_opt * dscale, p, cap, &iters, &degp);
        it1 = iters;
        if (r == OR_ITERATION_LIMIT) { status = r; goto done; }
        if (r == OR_UNBOUNDED) { status = OR_NUMERICAL; goto done; }
        const double wstar = -T_(&tb, m, tb.ncol);
        if (wstar < -p->tol_feas * (1.0 + bnorm)) { status = OR_INFEASIBLE; goto done; }
        /* Drive basic artificials out, in row order. */
        for (int i = 0; i < m; ++i) {
            if (!tb.is_art[tb.basis[i]])
                continue;
            int e = -1;
            for (int j = 0; j < tb.ncol; ++j) {
                if (tb.is_basic[j] || tb.is_art[j])
                    continue;
                if (fabs(T_(&tb, i, j)) > p->tol_piv) { e = j; break; }
            }
            if (e >= 0)
                pivot(&tb, i, e);
            else
                tb.row_dead[i] = 1;
        }
        for (int j = 0; j < tb.ncol; ++j)
            if (tb.is_art[j])
                tb.col_dead[j] = 1;
    }

    /* 5. Phase II. */
    for (int j = 0; j < tb.ncol; ++j)
        cost[j] = (j < n) ? c[j] : 0.0;
    price_out(&tb, cost);
    {
        int r = simplex_loop(&tb, p->tol_opt * (cnorm > 1.0 ? cnorm : 1.0), p, cap, &iters, &degp);
        if (r != OR_OPTIMAL) { status = r; goto done; }
    }

    /* 7. Extraction. */
    for (int j = 0; j < n; ++j)
        x[j] = 0.0;
    for (int i = 0; i < m; ++i)
        if (!tb.row_dead[i] && tb.basis[i] < n)
            x[tb.basis[i]] = T_(&tb, i, tb.ncol);
    {
        double z = 0.0;
        for (int j = 0; j < n; ++j)
            z = z + c[j] * x[j];
        *obj_out = z;
    }
done:
    if (status == OR_UNBOUNDED)
        *obj_out = INFINITY;
    if (status != OR_OPTIMAL)
        for (int j = 0; j < n; ++j)
            x[j] = NAN;
    if (basis_out)
        for (int i = 0; i < m; ++i)
            basis_out[i] = tb.row_dead[i] ? -1 : tb.bland[tb.basis[i]];
    if (stats) {
        stats[0] = it1;
        stats[1] = iters - it1;
        stats[2] = degp;
    }
    free(cost); free(sgn); free(sen);
    free(tb.t); free(tb.basis); free(tb.is_basic); free(tb.is_art);
    free(tb.col_dead); free(tb.row_dead); free(tb.bland);
    return status;
}

int oracle_solve_one(int m, int n, const double *A, const double *b, const double *c,
                     const int8_t *sense, const oracle_params *p,
                     double *x, double *obj_out, int32_t *basis_out, int32_t *stats)
{
    return solve_impl(m, n, A, b, c, sense, p, x, obj_out, basis_out, stats, NULL, NULL);
}

/* As oracle_solve_one, also recording the whole tableau after every pricing of
 * an objective row and after every pivot (at most trace_cap snapshots of
 * (m+1) x (ncol+1) doubles, objective row last).  *ncol receives the number of
 * variable columns and *nsnap the number of snapshots taken. */
int oracle_solve_traced(int m, int n, const double *A, const double *b, const double *c,
                        const int8_t *sense, const oracle_params *p,
                        double *x, double *obj_out, int32_t *basis_out, int32_t *stats,
                        double *trace_buf, int trace_cap, int32_t *ncol, int32_t *nsnap)
{
    trace_rec tr = { trace_buf, trace_cap, 0 };
    int nc = 0;
    int st = solve_impl(m, n, A, b, c, sense, p, x, obj_out, basis_out, stats, &tr, &nc);
    *ncol = nc;
    *nsnap = tr.count;
    return st;
}

/* ---- batch driver: a pthread pool handing out LPs dynamically ------------- */

typedef struct {
    int64_t num_lps;
    const double *A, *b, *c;
    const int8_t *sense;
    const int32_t *m, *n;
    const int64_t *aoff, *roff, *coff;
    const oracle_params *p;
    int32_t *status;
    double *x, *obj;
    int32_t *basis, *stats;
    int64_t next;
    pthread_mutex_t mu;
} batch_job;

static void *worker(void *arg)
{
    batch_job *jb = (batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&jb->mu);
        int64_t k = jb->next++;
        pthread_mutex_unlock(&jb->mu);
        if (k >= jb->num_lps)
            break;
        jb->status[k] = oracle_solve_one(
            jb->m[k], jb->n[k], jb->A + jb->aoff[k], jb->b + jb->roff[k], jb->c + jb->coff[k],
            jb->sense + jb->roff[k], jb->p, jb->x + jb->coff[k], jb->obj + k,
            jb->basis ? jb->basis + jb->roff[k] : NULL, jb->stats ? jb->stats + 3 * k : NULL);
    }
    return NULL;
}

/* Solves num_lps LPs stored back to back (A row-major per LP).  All arrays are
 * host memory owned by the caller.  nthreads <= 0 means one thread.
 * Returns 0, or -1 on a bad argument. */
int oracle_solve_batch(int64_t num_lps, const double *A, const double *b, const double *c,
                       const int8_t *sense, const int32_t *m, const int32_t *n,
                       const oracle_params *p, int nthreads,
                       int32_t *status, double *x, double *obj, int32_t *basis, int32_t *stats)
{
    if (num_lps < 0 || !p || !status || !x || !obj || !m || !n)
        return -1;
    batch_job jb;
    jb.aoff = malloc(sizeof(int64_t) * (num_lps + 1));
    jb.roff = malloc(sizeof(int64_t) * (num_lps + 1));
    jb.coff = malloc(sizeof(int64_t) * (num_lps + 1));
    int64_t sa = 0, sr = 0, sc = 0;
    for (int64_t k = 0; k < num_lps; ++k) {
        ((int64_t *)jb.aoff)[k] = sa; ((int64_t *)jb.roff)[k] = sr; ((int64_t *)jb.coff)[k] = sc;
        sa += (int64_t)m[k] * n[k]; sr += m[k]; sc += n[k];
    }
    jb.num_lps = num_lps; jb.A = A; jb.b = b; jb.c = c; jb.sense = sense; jb.m = m; jb.n = n;
    jb.p = p; jb.status = status; jb.x = x; jb.obj = obj; jb.basis = basis; jb.stats = stats;
    jb.next = 0;
    pthread_mutex_init(&jb.mu, NULL);
    if (nthreads < 1)
        nthreads = 1;
    pthread_t *th = malloc(sizeof(pthread_t) * nthreads);
    for (int t = 1; t < nthreads; ++t)
        pthread_create(&th[t], NULL, worker, &jb);
    worker(&jb);
    for (int t = 1; t < nthreads; ++t)
        pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&jb.mu);
    free((void *)jb.aoff); free((void *)jb.roff); free((void *)jb.coff);
    return 0;
}
