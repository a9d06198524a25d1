// certify_kernels.hip -- FP64 re-solve and certificate of a final basis.
//
// After a solve on a single-precision tableau, every LP's final basis is taken
// back to the FP64 input data:
//   * T = rows whose slack/surplus (or artificial) is non-basic ("tight"),
//     S = basic structural variables; |T| = |S| = k for a square basis.
//   * B_TS = the k x k block of the sign-normalised constraint matrix is
//     LU-factorised with partial pivoting;  x_S = B_TS^-1 b_T  (x_B = B^-1 b),
//     y_T = B_TS^-T c_S  (the duals, y = 0 on the other rows).
//   * Primal certificate: x_S >= -tol and every non-tight row's slack or
//     surplus >= -tol (a dropped redundant row's residual within tol).
//   * Dual certificate (reduced costs): c_j - y^T a_j <= tol for every
//     non-basic structural j, and for the logical of every tight row:
//     -y_i <= tol (slack, <= row) or y_i <= tol (surplus, >= row).
//     Together these give c^T x = b^T y, i.e. optimality (strong duality).
//   * For an LP reported unbounded with entering variable q: the ray
//     (x_q = t, x_S = x_S - t B^-1 a_q) must keep every basic variable and
//     every row's slack non-decreasing where it must stay non-negative and
//     raise the objective, and the LP must have a feasible point: the basis
//     passes the primal certificate, or x = 0 is feasible (every normalised
//     row is <= or has b = 0), as for LPs whose rows are all <= with b >= 0.
//   * For an LP reported infeasible (workgroup kernel, LPs with their own
//     constraints): the final basis is the Phase I basis (artificial cost -1,
//     rows R whose artificial is basic).  x_S = B_TS^-1 b_T, every artificial
//     and slack value >= -tol, y_T = B_TS^-T (sum over R of the rows' entries
//     in S), y = -1 on R; every structural and slack / surplus reduced cost
//     <= tol (artificials are not priced again once they left); and the Phase
//     I optimum w* = -(sum of the artificial values) below -tol.  -y is then
//     a Farkas certificate of infeasibility.
// An LP whose result passes is written with its FP64 x and objective (an
// unbounded one with x = NaN and +inf; an infeasible one keeps the solve's
// NaN outputs); any other
// LP (failed certificate, singular block, or a status the kernel does not
// certify) is appended to the fallback list for the FP64 re-solve, which
// starts from the single-precision final basis where it can.
#include <math.h>

#include "device_common.h"
#include "internal.h"

namespace lpb {
namespace {

constexpr int kTight = 32, kDeadRow = 64, kArtRow = 128;

template <int NT>
struct CertCtrl {
    int k, kt, fail, next;
    int piv;
    int pad[3];
    double bnorm, cnorm, amax;
    double rd[16];
    int ri[16];
};

template <int NT>
__device__ __forceinline__ double blk_max(double v, CertCtrl<NT> *sh)
{
    v = wave_max_f(v);
    if constexpr (NT > 64) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) sh->rd[w] = v;
        __syncthreads();
        v = sh->rd[0];
#pragma unroll
        for (int q = 1; q < NT / 64; ++q) v = fmax(v, sh->rd[q]);
        __syncthreads();
    }
    return v;
}

// Largest key over the block, ties to the smallest index (key >= 0, idx unique).
template <int NT>
__device__ __forceinline__ void blk_argmax(double &key, int &idx, CertCtrl<NT> *sh)
{
    {
        // Within the wavefront: DPP / permlane reductions and a ballot.
        const double best = wave_max_f(key);
        const int imin = wave_min_i(key == best ? idx : kBig);
        key = best;
        idx = imin;
    }
    if constexpr (NT > 64) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) { sh->rd[w] = key; sh->ri[w] = idx; }
        __syncthreads();
        key = sh->rd[0]; idx = sh->ri[0];
#pragma unroll
        for (int q = 1; q < NT / 64; ++q) {
            const double ok = sh->rd[q];
            const int oi = sh->ri[q];
            if (ok > key || (ok == key && oi < idx)) { key = ok; idx = oi; }
        }
        __syncthreads();
    }
}

// Compacts the flagged entries of [0, count) into list (ascending); wave 0 only.
__device__ __forceinline__ int compact(const int *flag, int mask, int count, int *list, int *pos,
                                      int cap = 0x7fffffff)
{
    const int lane = threadIdx.x & 63;
    int base = 0;
    for (int i0 = 0; i0 < count; i0 += 64) {
        const int i = i0 + lane;
        const bool on = i < count && (flag[i] & mask);
        const uint64_t b = __ballot(on);
        if (on) {
            const int p = base + __popcll(b & lanemask_lt(lane));
            if (p < cap) list[p] = i;  // a list holds cap entries; the count goes on
            pos[i] = p;
        } else if (i < count) {
            pos[i] = -1;
        }
        base += __popcll(b);
    }
    return base;
}

template <int NT>
__global__ __launch_bounds__(NT) void certify_kernel(CertArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    CertCtrl<NT> *sh = reinterpret_cast<CertCtrl<NT> *>(smem);
    const int64_t total = a.num;
    int64_t item = blockIdx.x;
    while (item < total) {
        if (tid == 0) sh->next = int(gridDim.x) + atomicAdd(a.queue, 1);
        const int64_t k = !a.order1 ? item : (item < a.n1 ? a.order1[item] : a.order2[item - a.n1]);
        int m, n;
        int64_t ao, ro, co;
        if (a.um > 0) {
            m = a.um; n = a.un; ao = k * int64_t(m) * n; ro = k * m; co = k * n;
        } else {
            m = a.m[k]; n = a.n[k]; ao = a.aoff[k]; ro = a.roff[k]; co = a.coff[k];
        }
        const double *A = a.A + ao, *b = a.b + ro, *c = a.c + co;
        const int8_t *sense = a.sense + ro;
        const int32_t *basis = a.basis + ro;
        // Screened solve: the basis covers the ms rows sub[] of the shared LP
        // (in that solve's numbering); every other row's slack is basic.
        const int32_t *sub = nullptr;
        int ms = m;
        if (a.shared) {
            A = a.A;
            b = a.b;
            sense = a.sense;
            if (a.row_subset) {
                ms = a.subset_m;
                sub = a.row_subset + k * int64_t(ms);
                basis = a.basis + k * int64_t(ms);
            }
        }
        double *x = a.x + co;
        const int st0 = a.status[k];
        // LDS carve-up for this LP.
        int *rowf = reinterpret_cast<int *>(smem + align16(sizeof(CertCtrl<NT>)));
        int *tpos = rowf + m;
        int *tlist = tpos + m;
        int *colf = tlist + m;
        int *spos = colf + n;
        int *slist = spos + n;
        double *vec = reinterpret_cast<double *>(smem + align16(sizeof(CertCtrl<NT>)) +
                                                 align16(4 * int64_t(3 * m + 3 * n)));
        const int kmax = min(m, n);
        double *xs = vec;           // [kmax] x_S, then scratch
        double *yt = xs + kmax;     // [kmax] y_T
        double *wv = yt + kmax;     // [kmax] ray direction
        int *perm = reinterpret_cast<int *>(wv + kmax);  // [kmax] row permutation of the LU
        const int64_t mat_off = align16(sizeof(CertCtrl<NT>)) + align16(4 * int64_t(3 * m + 3 * n)) +
                                align16(8 * 3 * int64_t(kmax) + 4 * int64_t(kmax));
        int cert = 0;
        // An infeasible result of an LP's own constraints: the Phase I
        // certificate (a screened relaxation's goes to the re-solve).
        const bool phase1 = st0 == kInfeasible && !sub;
        bool fallback = !(st0 == kOptimal || st0 == kUnbounded || phase1);
        // Invalid input stays invalid -- unless it was only the screening's row
        // list that was bad: the re-solve on all rows then decides.
        if (st0 == kInvalid) fallback = a.shared && a.row_subset;
        const bool work = st0 == kOptimal || st0 == kUnbounded || phase1;
        bool origin_out = false;  // this thread's rows: is x = 0 outside the feasible set?

        if (work) {
            // Rows: sign normalisation, and which rows are tight.
            if (tid == 0) sh->fail = 0;
            for (int i = tid; i < m; i += NT) {
                const double bi = b[i];
                int sen = sense[i];
                const bool neg = bi < 0.0;
                if (neg && sen != kEQ) sen = (sen == kLE) ? kGE : kLE;
                rowf[i] = (neg ? kRowNeg : 0) | (sen << 1) | (sub ? 0 : kTight);
                origin_out |= sen != kLE && bi != 0.0;
            }
            for (int j = tid; j < n; j += NT) colf[j] = 0;
            __syncthreads();
            // Row of the full LP behind row r of the solve that made the basis.
            auto full_row = [&](int r) -> int {
                if (!sub) return r;
                const int q = sub[r];
                return (q >= 0 && q < m) ? q : -1;
            };
            if (sub) {
                for (int r = tid; r < ms; r += NT) {
                    const int q = full_row(r);
                    if (q < 0) sh->fail = 9;
                    else atomicOr(&rowf[q], kTight);
                }
                __syncthreads();
            }
            for (int r = tid; r < ms; r += NT) {
                const int v = basis[r];
                if (v < -1 || v >= n + 2 * ms) {
                    sh->fail = 9;  // not a basis of this LP
                } else if (v < 0) {
                    const int q = full_row(r);
                    if (q < 0) { sh->fail = 9; continue; }
                    atomicOr(&rowf[q], kDeadRow);
                    atomicAnd(&rowf[q], ~kTight);
                } else if (v < n) {
                    colf[v] = kTight;
                } else if (v < n + ms) {
                    const int q = full_row(v - n);
                    if (q < 0) { sh->fail = 9; continue; }
                    atomicAnd(&rowf[q], ~kTight);
                } else {
                    // A basic artificial: a redundant row at an optimum, a row
                    // of the Phase I objective at an infeasible end.
                    const int q = full_row(v - n - ms);
                    if (q < 0) { sh->fail = 9; continue; }
                    atomicOr(&rowf[q], phase1 ? kArtRow : kDeadRow);
                    atomicAnd(&rowf[q], ~kTight);
                }
            }
            __syncthreads();
            if (wave == 0) {
                const int kt = compact(rowf, kTight, m, tlist, tpos);
                const int ks = compact(colf, kTight, n, slist, spos);
                if (lane == 0) { sh->kt = kt; sh->k = ks; }
            }
            double bm = 0.0, cm = 0.0;
            for (int i = tid; i < m; i += NT) bm = fmax(bm, fabs(b[i]));
            for (int j = tid; j < n; j += NT) cm = fmax(cm, fabs(c[j]));
            __syncthreads();
            const double bnorm = blk_max<NT>(bm, sh), cnorm = blk_max<NT>(cm, sh);
            const int K = sh->k;
            const double tol_p = a.tol_feas * (1.0 + bnorm);
            const double tol_d = a.tol_opt * fmax(1.0, cnorm);
            bool ok = sh->kt == K && sh->fail == 0;
            double *M = nullptr;
            if (ok) {
                M = (mat_off + 8 * int64_t(K) * K <= a.lds_bytes)
                        ? reinterpret_cast<double *>(smem + mat_off)
                        : reinterpret_cast<double *>(a.scratch + int64_t(blockIdx.x) * a.slot_bytes);
                // B_TS, row-major K x K, sign-normalised: thread columns s2,
                // rows in groups of 8 whose loads precede their stores.
                for (int s2 = tid; s2 < K; s2 += NT) {
                    const int jc = slist[s2];
                    for (int t0 = 0; t0 < K; t0 += 8) {
                        double v[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int t = t0 + q;
                            if (t < K) {
                                const int i = tlist[t];
                                v[q] = ((rowf[i] & kRowNeg) ? -1.0 : 1.0) * A[int64_t(i) * n + jc];
                            }
                        }
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            if (t0 + q < K) M[(t0 + q) * K + s2] = v[q];
                    }
                }
                for (int t = tid; t < K; t += NT) {
                    const int i = tlist[t];
                    xs[t] = ((rowf[i] & kRowNeg) ? -1.0 : 1.0) * b[i];
                    double ct = 0.0;
                    if (phase1) {
                        // c_S = 0 and y = -1 on the artificials' rows R:
                        // B_TS^T y_T = sum over R of the rows' entries in S.
                        const int jc = slist[t];
                        for (int r2 = 0; r2 < m; ++r2)
                            if (rowf[r2] & kArtRow)
                                ct += ((rowf[r2] & kRowNeg) ? -1.0 : 1.0) * A[int64_t(r2) * n + jc];
                    } else {
                        ct = c[slist[t]];
                    }
                    yt[t] = ct;
                    perm[t] = t;
                }
                double am = 0.0;
                for (int e = tid; e < K * K; e += NT) am = fmax(am, fabs(M[e]));
                __syncthreads();
                const double amax = blk_max<NT>(am, sh);
                // LU with partial pivoting (ties to the smaller row).  Column p
                // of each step is copied into LDS (colb) by the pivot search,
                // scaled there into the multipliers and read back by the
                // trailing update, so a block in device memory is read for its
                // entries and its swapped rows only.
                double *colb = wv;  // [kmax], free until the ray check
                for (int p = 0; p < K; ++p) {
                    double key = -1.0;
                    int idx = kBig;
                    for (int i = p + tid; i < K; i += NT) {
                        const double cv = M[i * K + p];
                        colb[i] = cv;
                        const double v = fabs(cv);
                        if (v > key || (v == key && i < idx)) { key = v; idx = i; }
                    }
                    blk_argmax<NT>(key, idx, sh);
                    if (!(key > 1e-13 * fmax(1.0, amax))) { ok = false; break; }
                    if (idx != p) {
                        for (int j = tid; j < K; j += NT) {
                            const double t0 = M[p * K + j];
                            M[p * K + j] = M[idx * K + j];
                            M[idx * K + j] = t0;
                        }
                        if (tid == 0) {
                            const double t1 = xs[p]; xs[p] = xs[idx]; xs[idx] = t1;
                            const int t2 = perm[p]; perm[p] = perm[idx]; perm[idx] = t2;
                            const double t3 = colb[p]; colb[p] = colb[idx]; colb[idx] = t3;
                        }
                    }
                    __syncthreads();
                    const double inv = 1.0 / colb[p];
                    for (int i = p + 1 + tid; i < K; i += NT) {
                        const double l = colb[i] * inv;
                        M[i * K + p] = l;
                        colb[i] = l;
                    }
                    __syncthreads();
                    // Trailing update: thread (r0, c0) takes column p+1+c0 of
                    // rows p+1+r0, p+1+r0+rpp, ... (one division per step, not
                    // per entry; consecutive threads on consecutive columns).
                    // Rows go in groups of LB whose loads are all issued before
                    // any store (the compiler may not move a load past a possibly
                    // aliasing store), so a block in device memory costs one round
                    // trip per group rather than one per row.
                    const int rem = K - p - 1;
                    constexpr int LB = 16;
                    auto update_column = [&](int j, int i_first, int di) {
                        const double upj = M[p * K + j];
                        for (int i0 = i_first; i0 < K; i0 += LB * di) {
                            double mv[LB];
#pragma unroll
                            for (int q = 0; q < LB; ++q) {
                                const int i = i0 + q * di;
                                if (i < K) mv[q] = M[i * K + j];
                            }
#pragma unroll
                            for (int q = 0; q < LB; ++q) {
                                const int i = i0 + q * di;
                                if (i < K) M[i * K + j] = fma(-colb[i], upj, mv[q]);
                            }
                        }
                    };
                    if (rem == 0) {
                        // last step: nothing below the pivot
                    } else if (rem <= NT) {
                        const int rpp = NT / rem;
                        if (tid < rpp * rem) {
                            const int r0 = tid / rem;
                            update_column(p + 1 + (tid - r0 * rem), p + 1 + r0, rpp);
                        }
                    } else {
                        for (int j = p + 1 + tid; j < K; j += NT) update_column(j, p + 1, 1);
                    }
                    __syncthreads();
                }
                if (!ok) cert |= LP_CERT_SINGULAR_BIT;
            }
            if (ok) {
                // x_S: L z = P b_T (xs already permuted), U x = z.
                for (int p = 0; p < K; ++p) {
                    const double zp = xs[p];
                    for (int i = p + 1 + tid; i < K; i += NT) xs[i] = fma(-M[i * K + p], zp, xs[i]);
                    __syncthreads();
                }
                for (int p = K - 1; p >= 0; --p) {
                    const double xp = xs[p] / M[p * K + p];
                    __syncthreads();
                    if (tid == 0) xs[p] = xp;
                    for (int i = tid; i < p; i += NT) xs[i] = fma(-M[i * K + p], xp, xs[i]);
                    __syncthreads();
                }
                // y_T: B^T y = c_S  ->  U^T w = c_S, L^T v = w, y = P^T v.
                for (int p = 0; p < K; ++p) {
                    const double wp = yt[p] / M[p * K + p];
                    __syncthreads();
                    if (tid == 0) yt[p] = wp;
                    for (int j = p + 1 + tid; j < K; j += NT) yt[j] = fma(-M[p * K + j], wp, yt[j]);
                    __syncthreads();
                }
                for (int p = K - 1; p >= 0; --p) {
                    const double vp = yt[p];
                    for (int j = tid; j < p; j += NT) yt[j] = fma(-M[p * K + j], vp, yt[j]);
                    __syncthreads();
                }
                // Undo the row permutation: y for tight row tlist[perm[p]] is yt[p].
                for (int p = tid; p < K; p += NT) wv[perm[p]] = yt[p];
                __syncthreads();
                for (int p = tid; p < K; p += NT) yt[p] = wv[p];
                __syncthreads();

                // Primal certificate.
                bool pf = true;
                double art = 0.0;  // Phase I: this thread's artificial values
                for (int s2 = tid; s2 < K; s2 += NT) pf &= xs[s2] >= -tol_p;
                for (int i = tid; i < m; i += NT) {
                    const int f = rowf[i];
                    if (f & kTight) continue;
                    const double sg = (f & kRowNeg) ? -1.0 : 1.0;
                    double ax = 0.0;
                    for (int s2 = 0; s2 < K; ++s2) ax = fma(A[int64_t(i) * n + slist[s2]], xs[s2], ax);
                    const double r = sg * (b[i] - ax);  // normalised slack b_i - a_i x
                    const int sen = (f >> 1) & 3;
                    if (f & kArtRow) { pf &= r >= -tol_p; art += r; }  // the row's artificial value
                    else if ((f & kDeadRow) || sen == kEQ) pf &= fabs(r) <= tol_p;  // a row left out of a screened solve can be an equality
                    else if (sen == kLE) pf &= r >= -tol_p;
                    else if (sen == kGE) pf &= -r >= -tol_p;
                }
                if (!pf) sh->fail = 1;
                __syncthreads();
                const bool primal_ok = sh->fail == 0;
                if (primal_ok) cert |= LP_CERT_PRIMAL_OK_BIT;
                __syncthreads();

                if (phase1 && primal_ok) {
                    // Phase I optimum w* = -(sum of the artificial values), the
                    // largest reduced cost 0 - y^T a_j over the non-basic
                    // structurals (y = y_T on T, -1 on R) and the scale of
                    // Phase I's first objective row (the sums over the >= and
                    // = rows), each reduced over the workgroup.
                    double worst = -1.0, dmax = 1.0;
                    for (int j = tid; j < n; j += NT) {
                        double start = 0.0, onr = 0.0;
                        for (int i = 0; i < m; ++i) {
                            const int f = rowf[i];
                            const double v = ((f & kRowNeg) ? -1.0 : 1.0) * A[int64_t(i) * n + j];
                            if (((f >> 1) & 3) != kLE) start += v;
                            if (f & kArtRow) onr += v;
                        }
                        dmax = fmax(dmax, fabs(start));
                        if (spos[j] >= 0) continue;
                        double ya = 0.0;
                        for (int t = 0; t < K; ++t) {
                            const int i = tlist[t];
                            const double sg = (rowf[i] & kRowNeg) ? -1.0 : 1.0;
                            ya = fma(yt[t], sg * A[int64_t(i) * n + j], ya);
                        }
                        worst = fmax(worst, onr - ya);  // -(y_T^T a_Tj - a_Rj)
                    }
                    // Slacks / surpluses of the tight rows (cost 0): -sigma_i y_i.
                    for (int t = tid; t < K; t += NT) {
                        const int sen = (rowf[tlist[t]] >> 1) & 3;
                        if (sen == kLE) worst = fmax(worst, -yt[t]);
                        else if (sen == kGE) worst = fmax(worst, yt[t]);
                    }
                    double wsum = art;
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off);
                    if constexpr (NT > 64) {
                        if (lane == 0) sh->rd[wave] = wsum;
                        __syncthreads();
                        wsum = 0.0;
                        for (int qq = 0; qq < NT / 64; ++qq) wsum += sh->rd[qq];
                        __syncthreads();
                    }
                    worst = blk_max<NT>(worst, sh);
                    dmax = blk_max<NT>(dmax, sh);
                    const double wstar = -wsum;
                    if (worst <= a.tol_opt * dmax && wstar < -tol_p) cert |= LP_CERT_INFEASIBLE_OK_BIT;
                }
                if (st0 == kOptimal && primal_ok) {
                    // Dual certificate: reduced costs of every non-basic column.
                    bool df = true;
                    for (int j = tid; j < n; j += NT) {
                        if (spos[j] >= 0) continue;
                        double ya = 0.0;
                        for (int t = 0; t < K; ++t) {
                            const int i = tlist[t];
                            const double sg = (rowf[i] & kRowNeg) ? -1.0 : 1.0;
                            ya = fma(yt[t], sg * A[int64_t(i) * n + j], ya);
                        }
                        df &= c[j] - ya <= tol_d;
                    }
                    for (int t = tid; t < K; t += NT) {
                        const int sen = (rowf[tlist[t]] >> 1) & 3;
                        if (sen == kLE) df &= -yt[t] <= tol_d;
                        else if (sen == kGE) df &= yt[t] <= tol_d;
                    }
                    if (!df) sh->fail = 2;
                    __syncthreads();
                    if (sh->fail == 0) cert |= LP_CERT_DUAL_OK_BIT;
                }
                // x = 0 is feasible when every normalised row is <= (b >= 0) or
                // has b = 0: then a ray alone proves the LP unbounded, whatever
                // the FP64 values of the final basis.
                const bool origin = blk_max<NT>(origin_out ? 1.0 : 0.0, sh) == 0.0;
                if (st0 == kUnbounded && (primal_ok || origin)) {
                    // Ray of the entering variable q.
                    if (tid == 0) sh->fail = 0;  // a failed primal check is not the ray's
                    __syncthreads();
                    int q = a.enter[k];
                    if (sub && q >= n && q < n + ms) {
                        const int fr = full_row(q - n);
                        q = fr >= 0 ? n + fr : -1;
                    } else if (sub && q >= n + ms) {
                        q = -1;
                    }
                    bool rf = q >= 0 && q < n + m && !(q < n && spos[q] >= 0);
                    int tr = -1;
                    double sq = 0.0;
                    if (rf && q >= n) {
                        tr = tpos[q - n];
                        const int sen = (rowf[q - n] >> 1) & 3;
                        rf = tr >= 0 && sen != kEQ;
                        sq = (sen == kLE) ? 1.0 : -1.0;
                    }
                    if (rf) {
                        // wv = B^-1 a_q restricted to T (then d_S = -wv).
                        for (int t = tid; t < K; t += NT) {
                            const int i = tlist[t];
                            const double sg = (rowf[i] & kRowNeg) ? -1.0 : 1.0;
                            yt[t] = (q < n) ? sg * A[int64_t(i) * n + q] : (t == tr ? sq : 0.0);
                        }
                        __syncthreads();
                        if (tid == 0)
                            for (int p = 0; p < K; ++p) {  // apply the row permutation
                                wv[p] = yt[perm[p]];
                            }
                        __syncthreads();
                        for (int p = 0; p < K; ++p) {
                            const double zp = wv[p];
                            for (int i = p + 1 + tid; i < K; i += NT) wv[i] = fma(-M[i * K + p], zp, wv[i]);
                            __syncthreads();
                        }
                        for (int p = K - 1; p >= 0; --p) {
                            const double xp = wv[p] / M[p * K + p];
                            __syncthreads();
                            if (tid == 0) wv[p] = xp;
                            for (int i = tid; i < p; i += NT) wv[i] = fma(-M[i * K + p], xp, wv[i]);
                            __syncthreads();
                        }
                        const double tol_r = a.tol_feas;
                        bool ok2 = true;
                        double gain = 0.0;
                        for (int s2 = tid; s2 < K; s2 += NT) {
                            ok2 &= -wv[s2] >= -tol_r;
                            gain = fma(c[slist[s2]], -wv[s2], gain);
                        }
                        for (int i = tid; i < m; i += NT) {
                            const int f = rowf[i];
                            if (f & kTight) continue;
                            const double sg = (f & kRowNeg) ? -1.0 : 1.0;
                            double ad = (q < n) ? A[int64_t(i) * n + q] : 0.0;
                            for (int s2 = 0; s2 < K; ++s2) ad = fma(A[int64_t(i) * n + slist[s2]], -wv[s2], ad);
                            const double dr = -sg * ad;  // change of the normalised slack
                            const int sen = (f >> 1) & 3;
                            if ((f & kDeadRow) || sen == kEQ) ok2 &= fabs(dr) <= tol_r;
                            else if (sen == kLE) ok2 &= dr >= -tol_r;
                            else if (sen == kGE) ok2 &= -dr >= -tol_r;
                        }
                        if (!ok2) sh->fail = 3;
                        double g = gain;
#pragma unroll
                        for (int off = 32; off > 0; off >>= 1) g += __shfl_xor(g, off);
                        if constexpr (NT > 64) {
                            if (lane == 0) sh->rd[wave] = g;
                            __syncthreads();
                            g = 0.0;
                            for (int qq = 0; qq < NT / 64; ++qq) g += sh->rd[qq];
                        }
                        __syncthreads();
                        const double cq = (q < n) ? c[q] : 0.0;
                        if (sh->fail == 0 && cq + g > tol_d) cert |= LP_CERT_RAY_OK_BIT;
                        __syncthreads();
                    }
                }
            }
            const bool passed = phase1 ? (cert & LP_CERT_INFEASIBLE_OK_BIT) != 0
                                : (st0 == kOptimal) ? (cert & LP_CERT_DUAL_OK_BIT) && (cert & LP_CERT_PRIMAL_OK_BIT)
                                                    : (cert & LP_CERT_RAY_OK_BIT) != 0;
            fallback = !passed;
            if (passed && st0 == kOptimal) {
                // FP64 x and objective (fixed summation order by wavefront 0).
                for (int j = tid; j < n; j += NT) x[j] = (spos[j] >= 0) ? xs[spos[j]] : 0.0;
                if (wave == 0) {
                    double z = 0.0;
                    for (int j = lane; j < n; j += 64) z = fma(c[j], (spos[j] >= 0) ? xs[spos[j]] : 0.0, z);
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) z += __shfl_xor(z, off);
                    if (lane == 0) a.obj[k] = z;
                }
            } else if (passed && st0 == kUnbounded) {
                for (int j = tid; j < n; j += NT) x[j] = __builtin_nan("");
                if (tid == 0) a.obj[k] = __builtin_inf();
            }
        }
        if (tid == 0) {
            if (a.stats) a.stats[8 * k + 5] = cert;
            if (fallback) {
                const int slot = atomicAdd(a.fb_count, 1);
                a.fb_ids[slot] = int32_t(k);
            }
        }
        __syncthreads();
        item = sh->next;
        __syncthreads();
    }
    if (tid == 0) finish_launch(a.queue, a.done, nullptr);
}


// Compiler-level ordering point for a wavefront's own LDS traffic: the
// hardware keeps one wavefront's LDS accesses in program order, so a fence at
// wavefront scope is all that keeps the compiler from reordering them.
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

__device__ __forceinline__ bool wave_all(bool v) { return __ballot(!v) == 0; }

// The same certificate with one wavefront per LP and no workgroup barrier:
// lane t holds row t of the k x k block B_TS (column-major in LDS), the LU
// picks each pivot by a wavefront max (ties to the lower lane) and records
// the order instead of swapping rows; triangular solves broadcast one value
// per step with readlane.  W wavefronts share a workgroup, each with its own
// LP and LDS region; with stage_a the shared constraint matrix is copied into
// LDS once per workgroup and every A access of the certificate hits LDS.
template <int W, bool STAGE>
__global__ __launch_bounds__(64 * W) void certify_wave_kernel(CertArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // Entries loaded ahead per group: four when sixteen wavefronts share a
    // CU (128 VGPRs each), eight otherwise.
    constexpr int CG = W >= 16 ? 4 : 8;
    int64_t off = 0;
    if constexpr (STAGE) {
        // Rows at an odd stride of doubles: lanes reading one row each (the
        // LU's gather of B_TS, the primal check) then hit distinct banks.
        double *As = reinterpret_cast<double *>(smem);
        const int lds_n = a.un | 1;
        const int64_t cnt = int64_t(a.um) * a.un;
        for (int64_t e = threadIdx.x; e < cnt; e += 64 * W) As[(e / a.un) * lds_n + e % a.un] = a.A[e];
        __syncthreads();
        off = align16(8 * int64_t(a.um) * lds_n);
    }
    char *my = smem + off + int64_t(wave) * a.wave_bytes;
    const int64_t total = a.num;
    int64_t item = int64_t(blockIdx.x) * W + wave;
    while (item < total) {
        int nxt = 0;
        if (lane == 0) nxt = int(gridDim.x) * W + atomicAdd(a.queue, 1);
        const int64_t k = item;
        int m, n;
        int64_t ao, ro, co;
        if (a.um > 0) {
            m = a.um; n = a.un; ao = k * int64_t(m) * n; ro = k * m; co = k * n;
        } else {
            m = a.m[k]; n = a.n[k]; ao = a.aoff[k]; ro = a.roff[k]; co = a.coff[k];
        }
        // A stays in one address space per instantiation (LDS when staged),
        // so its loads compile to LDS or global instructions, not flat ones.
        const double *A = STAGE ? reinterpret_cast<const double *>(smem) : a.A + (a.shared ? 0 : ao);
        const int lda = STAGE ? (n | 1) : n;  // row stride of A
        const double *b = a.b + ro, *c = a.c + co;
        const int8_t *sense = a.sense + ro;
        const int32_t *basis = a.basis + ro;
        const int32_t *sub = nullptr;
        int ms = m;
        if (a.shared) {
            b = a.b;
            sense = a.sense;
            if (a.row_subset) {
                ms = a.subset_m;
                sub = a.row_subset + k * int64_t(ms);
                basis = a.basis + k * int64_t(ms);
            }
        }
        double *x = a.x + co;
        const int st0 = a.status[k];
        const WaveCertLayout L = wave_cert_layout(m, n, a.kl);
        int *rowf = reinterpret_cast<int *>(my + L.rowf);
        int *tpos = reinterpret_cast<int *>(my + L.tpos);
        int *colf = reinterpret_cast<int *>(my + L.colf);
        int *spos = reinterpret_cast<int *>(my + L.spos);
        int *tlist = reinterpret_cast<int *>(my + L.tlist);
        int *slist = reinterpret_cast<int *>(my + L.slist);
        int *order = reinterpret_cast<int *>(my + L.order);
        double *xsv = reinterpret_cast<double *>(my + L.xs);
        double *yv = reinterpret_cast<double *>(my + L.yv);
        int cert = 0;
        bool fallback = !(st0 == kOptimal || st0 == kUnbounded);
        if (st0 == kInvalid) fallback = a.shared && a.row_subset;
        const bool work = st0 == kOptimal || st0 == kUnbounded;
        if (a.viol && lane == 0) a.viol[k] = kBig;  // until the primal check counts them

        bool origin_out = false;  // this lane's rows: is x = 0 outside the feasible set?
        if (work) {
            // Rows: sign normalisation and the tight set; columns: the basic set.
            for (int i = lane; i < m; i += 64) {
                const double bi = b[i];
                int sen = sense[i];
                const bool neg = bi < 0.0;
                if (neg && sen != kEQ) sen = (sen == kLE) ? kGE : kLE;
                rowf[i] = (neg ? kRowNeg : 0) | (sen << 1) | (sub ? 0 : kTight);
                origin_out |= sen != kLE && bi != 0.0;
            }
            for (int j = lane; j < n; j += 64) colf[j] = 0;
            wave_sync();
            bool bad = false;
            auto full_row = [&](int r) -> int {
                if (!sub) return r;
                const int q = sub[r];
                return (q >= 0 && q < m) ? q : -1;
            };
            if (sub) {
                for (int r = lane; r < ms; r += 64) {
                    const int q = full_row(r);
                    if (q < 0) bad = true;
                    else atomicOr(&rowf[q], kTight);
                }
                wave_sync();
            }
            for (int r = lane; r < ms; r += 64) {
                const int v = basis[r];
                int q = -1;
                if (v < -1 || v >= n + 2 * ms) {
                    bad = true;
                } else if (v < 0) {
                    q = full_row(r);
                    if (q < 0) bad = true;
                    else { atomicOr(&rowf[q], kDeadRow); atomicAnd(&rowf[q], ~kTight); }
                } else if (v < n) {
                    colf[v] = kTight;
                } else if (v < n + ms) {
                    q = full_row(v - n);
                    if (q < 0) bad = true;
                    else atomicAnd(&rowf[q], ~kTight);
                } else {
                    q = full_row(v - n - ms);
                    if (q < 0) bad = true;
                    else { atomicOr(&rowf[q], kDeadRow); atomicAnd(&rowf[q], ~kTight); }
                }
            }
            wave_sync();
            // (Lists of 64 entries: more tight rows or basic structurals than
            // that fail the K <= kl test below.)
            // (Counts made wavefront-uniform for the compiler: loop bounds and
            // M's strides then live in scalar registers.)
            const int kt = uniform(compact(rowf, kTight, m, tlist, tpos, 64));
            const int K = uniform(compact(colf, kTight, n, slist, spos, 64));
            const int KL = K | 1;  // M's column stride: odd, so row reads of M miss no bank twice
            wave_sync();
            double bm = 0.0, cm = 0.0;
            for (int i = lane; i < m; i += 64) bm = fmax(bm, fabs(b[i]));
            for (int j = lane; j < n; j += 64) cm = fmax(cm, fabs(c[j]));
            const double bnorm = wave_max_f(bm), cnorm = wave_max_f(cm);
            const double tol_p = a.tol_feas * (1.0 + bnorm);
            const double tol_d = a.tol_opt * fmax(1.0, cnorm);
            // A basis with more than kl basic structurals (rare: the host sizes kl
            // for the batch) is left to the FP64 re-solve.
            bool ok = kt == K && K <= a.kl && __ballot(bad) == 0;
            double *M = reinterpret_cast<double *>(my + L.mat);
            // Lane t holds the t-th tight row (index and sign) and lane s the
            // s-th basic structural, so loops over T or S read them with
            // readlane instead of LDS.  M is B_TS column-major (M[s*KL + t],
            // row t in lane t); every loop over M loads CG entries ahead.
            const bool kfit = K <= a.kl;
            const int tl = (lane < K && kfit) ? tlist[lane] : 0;
            const int sl = (lane < K && kfit) ? slist[lane] : 0;
            const double sgt = (lane < K && kfit && (rowf[tl] & kRowNeg)) ? -1.0 : 1.0;
            double rz = 0.0, cs = 0.0;
            int pos = kBig;  // step at which this lane's row became the pivot row
            int ordr = 0;    // lane p: the row chosen at step p
            double rinv = 0.0;  // lane p: 1 / U_pp, recorded by the LU's step p
            if (ok) {
                double am = 0.0;
                // colv: this lane's entry of the column being eliminated, carried
                // in a register from the build and then from the previous step's
                // update; the pivot comes from its owner's register, so a step
                // reads only the pivot row and this lane's row segment from LDS.
                double colv = 0.0;
                const double *At = A + int64_t(tl) * lda;
                // (LDS and A reads are issued by the K lanes that own rows only:
                // their cost scales with the active lanes.)
                for (int s0 = 0; s0 < K; s0 += CG) {
                    int ci[CG];
#pragma unroll
                    for (int q = 0; q < CG; ++q) ci[q] = lane_get(sl, s0 + q < K ? s0 + q : 0);
                    double v[CG] = {};
                    if (lane < K) {
#pragma unroll
                        for (int q = 0; q < CG; ++q) v[q] = (s0 + q < K) ? sgt * At[ci[q]] : 0.0;
                    }
                    if (s0 == 0) colv = (lane < K) ? v[0] : 0.0;
#pragma unroll
                    for (int q = 0; q < CG; ++q)
                        if (s0 + q < K && lane < K) {
                            M[(s0 + q) * KL + lane] = v[q];
                            am = fmax(am, fabs(v[q]));
                        }
                }
                rz = (lane < K) ? sgt * b[tl] : 0.0;
                cs = (lane < K) ? c[sl] : 0.0;
                const double amax = wave_max_f(am);
                wave_sync();
                for (int p = 0; p < K; ++p) {
                    const double v = (lane < K && pos == kBig) ? fabs(colv) : -1.0;
                    // Every lane's reciprocal, computed while the maximum is
                    // reduced: the pivot's is taken below, off the serial chain.
                    const double cinv = 1.0 / colv;
                    const double vmax = wave_max_f(v);
                    if (!(vmax > 1e-13 * fmax(1.0, amax))) { ok = false; break; }
                    const int pl = __builtin_ctzll(__ballot(v == vmax));
                    if (lane == pl) pos = p;
                    if (lane == p) ordr = pl;
                    if (lane == 0) order[p] = pl;
                    const double uinv = lane_get(cinv, pl);
                    if (lane == p) rinv = uinv;
                    const bool act = lane < K && pos == kBig;
                    const int la = act ? lane : pl;
                    const double l = colv * uinv;
                    if (act) M[p * KL + lane] = l;
                    double nextv = 0.0;
                    if (act) {
                        for (int j0 = p + 1; j0 < K; j0 += CG) {
                            double pr[CG], mr[CG];
#pragma unroll
                            for (int q = 0; q < CG; ++q) {
                                const int j = j0 + q < K ? j0 + q : K - 1;
                                pr[q] = M[j * KL + pl];
                                mr[q] = M[j * KL + la];
                            }
#pragma unroll
                            for (int q = 0; q < CG; ++q) {
                                const double u = fma(-l, pr[q], mr[q]);
                                if (j0 + q < K) M[(j0 + q) * KL + lane] = u;
                                if (q == 0 && j0 == p + 1) nextv = u;
                            }
                        }
                    }
                    colv = nextv;
                    wave_sync();
                }
                if (!ok) cert |= LP_CERT_SINGULAR_BIT;
            }
            double xr = 0.0;  // lane p: x of the p-th basic structural
            if (ok) {
                // x_S (L z = P b_T, then U x = z) and y_T (U^T w = c_S, then
                // L^T v = w, y_t = v[pos_t]) side by side, so the two chains of
                // dependent steps overlap; 1 / U_pp comes from the LU (lane p).
                double wr = 0.0;
                for (int p0 = 0; p0 < K; p0 += CG) {
                    double mv[CG] = {}, mu[CG] = {};
                    int op[CG];
#pragma unroll
                    for (int q = 0; q < CG; ++q) op[q] = lane_get(ordr, p0 + q < K ? p0 + q : K - 1);
                    if (lane < K) {
#pragma unroll
                        for (int q = 0; q < CG; ++q) {
                            const int p = p0 + q < K ? p0 + q : K - 1;
                            mv[q] = M[p * KL + lane];               // lane t: L[t][p] (rows below p)
                            mu[q] = M[lane * KL + op[q]];           // lane j: U[p][j]
                        }
                    }
#pragma unroll
                    for (int q = 0; q < CG; ++q) {
                        const int p = p0 + q;
                        if (p < K) {
                            const double zp = lane_get(rz, lane_get(ordr, p));
                            if (lane < K && pos > p) rz = fma(-mv[q], zp, rz);
                            const double wp = lane_get(cs, p) * lane_get(rinv, p);
                            if (lane == p) wr = wp;
                            if (lane > p && lane < K) cs = fma(-mu[q], wp, cs);
                        }
                    }
                }
                for (int h = K - 1; h >= 0; h -= CG) {
                    double mv[CG] = {}, ml[CG] = {};
                    int op[CG];
#pragma unroll
                    for (int q = 0; q < CG; ++q) op[q] = lane_get(ordr, h - q >= 0 ? h - q : 0);
                    if (lane < K) {
#pragma unroll
                        for (int q = 0; q < CG; ++q) {
                            const int p = h - q >= 0 ? h - q : 0;
                            mv[q] = M[p * KL + lane];               // lane t: U[pos_t][p]
                            ml[q] = M[lane * KL + op[q]];           // lane p': L[p][p']
                        }
                    }
#pragma unroll
                    for (int q = 0; q < CG; ++q) {
                        const int p = h - q;
                        if (p >= 0) {
                            const int pl = lane_get(ordr, p);
                            const double xp = lane_get(rz, pl) * lane_get(rinv, p);
                            if (lane == p) xr = xp;
                            if (lane < K && pos < p) rz = fma(-mv[q], xp, rz);
                            const double vq = lane_get(wr, p);
                            if (lane < p) wr = fma(-ml[q], vq, wr);
                        }
                    }
                }
                if (lane < K) xsv[lane] = xr;
                const double yt = __shfl(wr, pos < 64 ? pos : 0);
                const double ysg = yt * sgt;  // dual times the row's sign
                if (lane < K) yv[lane] = yt;
                wave_sync();

                // Primal certificate: every non-tight row's slack from x_S.
                bool pf = !(lane < K) || xr >= -tol_p;
                int nviol = __popcll(__ballot(!pf));  // rows (and basic variables) out of bounds
                for (int i0 = 0; i0 < m; i0 += 64) {
                    bool rowok = true;
                    const int i = i0 + lane;
                    const int f = (i < m) ? rowf[i] : kTight;
                    const bool act = !(f & kTight);
                    const double *Ai = A + int64_t(act ? i : 0) * lda;
                    double ax[4] = {0.0, 0.0, 0.0, 0.0};
                    for (int s0 = 0; s0 < K; s0 += CG) {
                        int si[CG];
                        double xq[CG];
#pragma unroll
                        for (int q = 0; q < CG; ++q) {
                            si[q] = lane_get(sl, s0 + q < K ? s0 + q : 0);
                            xq[q] = lane_get(xr, s0 + q < K ? s0 + q : 0);
                        }
                        if (act) {  // only the rows that need the product read A
                            double av[CG];
#pragma unroll
                            for (int q = 0; q < CG; ++q) av[q] = Ai[si[q]];
#pragma unroll
                            for (int q = 0; q < CG; ++q)
                                if (s0 + q < K) ax[q & 3] = fma(av[q], xq[q], ax[q & 3]);
                        }
                    }
                    if (act) {
                        const double sg = (f & kRowNeg) ? -1.0 : 1.0;
                        const double r = sg * (b[i] - ((ax[0] + ax[1]) + (ax[2] + ax[3])));
                        const int sen = (f >> 1) & 3;
                        // A row left out of a screened solve can be an equality.
                        if ((f & kDeadRow) || sen == kEQ) rowok = fabs(r) <= tol_p;
                        else if (sen == kLE) rowok = r >= -tol_p;
                        else if (sen == kGE) rowok = -r >= -tol_p;
                    }
                    pf &= rowok;
                    nviol += __popcll(__ballot(!rowok));
                }
                const bool primal_ok = wave_all(pf);
                if (primal_ok) cert |= LP_CERT_PRIMAL_OK_BIT;
                if (a.viol && lane == 0) a.viol[k] = nviol;

                if (st0 == kOptimal && primal_ok) {
                    // Dual certificate: reduced costs of every non-basic column.
                    bool df = true;
                    for (int j0 = 0; j0 < n; j0 += 64) {
                        const int j = j0 + lane;
                        const bool act = j < n && spos[j] < 0;
                        const int jc = act ? j : 0;
                        double ya[4] = {0.0, 0.0, 0.0, 0.0};
                        for (int t0 = 0; t0 < K; t0 += CG) {
                            int ti[CG];
                            double yq[CG];
#pragma unroll
                            for (int q = 0; q < CG; ++q) {
                                ti[q] = lane_get(tl, t0 + q < K ? t0 + q : 0);
                                yq[q] = lane_get(ysg, t0 + q < K ? t0 + q : 0);
                            }
                            if (act) {  // only non-basic columns read A
                                double av[CG];
#pragma unroll
                                for (int q = 0; q < CG; ++q) av[q] = A[int64_t(ti[q]) * lda + jc];
#pragma unroll
                                for (int q = 0; q < CG; ++q)
                                    if (t0 + q < K) ya[q & 3] = fma(yq[q], av[q], ya[q & 3]);
                            }
                        }
                        if (act) df &= c[j] - ((ya[0] + ya[1]) + (ya[2] + ya[3])) <= tol_d;
                    }
                    if (lane < K) {
                        const int sen = (rowf[tl] >> 1) & 3;
                        if (sen == kLE) df &= -yt <= tol_d;
                        else if (sen == kGE) df &= yt <= tol_d;
                    }
                    if (wave_all(df)) cert |= LP_CERT_DUAL_OK_BIT;
                }
                // x = 0 feasible: the ray alone proves the LP unbounded.
                const bool origin = !__ballot(origin_out);
                if (st0 == kUnbounded && (primal_ok || origin)) {
                    // Ray of the entering variable q: w = B^-1 a_q, d_S = -w.
                    int q = a.enter[k];
                    if (sub && q >= n && q < n + ms) {
                        const int fr = full_row(q - n);
                        q = fr >= 0 ? n + fr : -1;
                    } else if (sub && q >= n + ms) {
                        q = -1;
                    }
                    bool rf = q >= 0 && q < n + m && !(q < n && spos[q] >= 0);
                    int tr = -1;
                    double sq = 0.0;
                    if (rf && q >= n) {
                        tr = tpos[q - n];
                        const int sen = (rowf[q - n] >> 1) & 3;
                        rf = tr >= 0 && sen != kEQ;
                        sq = (sen == kLE) ? 1.0 : -1.0;
                    }
                    if (rf) {
                        double rw = 0.0;
                        if (lane < K) {
                            const int i = tlist[lane];
                            const double sg = (rowf[i] & kRowNeg) ? -1.0 : 1.0;
                            rw = (q < n) ? sg * A[int64_t(i) * lda + q] : (lane == tr ? sq : 0.0);
                        }
                        for (int p = 0; p < K; ++p) {
                            const double zp = lane_get(rw, order[p]);
                            if (lane < K && pos > p) rw = fma(-M[p * KL + lane], zp, rw);
                        }
                        double wd = 0.0;
                        for (int p = K - 1; p >= 0; --p) {
                            const int pl = order[p];
                            const double xp = lane_get(rw, pl) / M[p * KL + pl];
                            if (lane == p) wd = xp;
                            if (lane < K && pos < p) rw = fma(-M[p * KL + lane], xp, rw);
                        }
                        const double tol_r = a.tol_feas;
                        bool ok2 = !(lane < K) || -wd >= -tol_r;
                        double gain = (lane < K) ? c[slist[lane]] * -wd : 0.0;
                        wave_sync();
                        if (lane < K) xsv[lane] = wd;  // x_S is no longer needed
                        wave_sync();
                        for (int i = lane; i < m; i += 64) {
                            const int f = rowf[i];
                            if (f & kTight) continue;
                            const double sg = (f & kRowNeg) ? -1.0 : 1.0;
                            double ad = (q < n) ? A[int64_t(i) * lda + q] : 0.0;
                            for (int s2 = 0; s2 < K; ++s2) ad = fma(A[int64_t(i) * lda + slist[s2]], -xsv[s2], ad);
                            const double dr = -sg * ad;
                            const int sen = (f >> 1) & 3;
                            if ((f & kDeadRow) || sen == kEQ) ok2 &= fabs(dr) <= tol_r;
                            else if (sen == kLE) ok2 &= dr >= -tol_r;
                            else if (sen == kGE) ok2 &= -dr >= -tol_r;
                        }
                        double g = gain;
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o);
                        const double cq = (q < n) ? c[q] : 0.0;
                        if (wave_all(ok2) && cq + g > tol_d) cert |= LP_CERT_RAY_OK_BIT;
                    }
                }
            }
            const bool passed = (st0 == kOptimal) ? (cert & LP_CERT_DUAL_OK_BIT) && (cert & LP_CERT_PRIMAL_OK_BIT)
                                                  : (cert & LP_CERT_RAY_OK_BIT) != 0;
            fallback = !passed;
            if (passed && st0 == kOptimal) {
                double z = 0.0;
                for (int j = lane; j < n; j += 64) {
                    const double xj = (spos[j] >= 0) ? xsv[spos[j]] : 0.0;
                    x[j] = xj;
                    z = fma(c[j], xj, z);
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) z += __shfl_xor(z, o);
                if (lane == 0) a.obj[k] = z;
            } else if (passed) {
                for (int j = lane; j < n; j += 64) x[j] = __builtin_nan("");
                if (lane == 0) a.obj[k] = __builtin_inf();
            }
        }
        if (lane == 0) {
            if (a.stats) a.stats[8 * k + 5] = cert;
            if (fallback) {
                const int slot = atomicAdd(a.fb_count, 1);
                a.fb_ids[slot] = int32_t(k);
            }
        }
        wave_sync();
        item = lane_get(nxt, 0);
    }
    __syncthreads();
    if (threadIdx.x == 0) finish_launch(a.queue, a.done, nullptr);
}

template <int NT>
hipError_t launch_t(const CertArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((certify_kernel<NT>), dim3(grid), dim3(NT), a.lds_bytes, s, a);
    return hipGetLastError();
}

template <int NT>
int occ_t(int lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void *)certify_kernel<NT>, NT, lds) !=
        hipSuccess)
        return 0;
    return blocks;
}

}  // namespace

int64_t certify_lds_bytes(int m, int n, bool with_matrix)
{
    const int kmax = m < n ? m : n;
    int64_t v = align16(sizeof(CertCtrl<256>)) + align16(4 * int64_t(3 * m + 3 * n)) +
                align16(8 * 3 * int64_t(kmax) + 4 * int64_t(kmax));
    if (with_matrix) v += 8 * int64_t(kmax) * kmax;
    return v;
}

hipError_t launch_certify(int nt, const CertArgs &a, int grid, hipStream_t s)
{
    return nt == 64 ? launch_t<64>(a, grid, s) : launch_t<256>(a, grid, s);
}

int certify_blocks_per_cu(int nt, int lds) { return nt == 64 ? occ_t<64>(lds) : occ_t<256>(lds); }

namespace {
template <int W, bool STAGE>
hipError_t launch_w(const CertArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((certify_wave_kernel<W, STAGE>), dim3(grid), dim3(64 * W), a.lds_bytes, s, a);
    return hipGetLastError();
}

template <int W, bool STAGE>
int occ_w(int lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void *)certify_wave_kernel<W, STAGE>, 64 * W,
                                                     lds) != hipSuccess)
        return 0;
    return blocks;
}
}  // namespace

// waves = 1: A read from device memory; 8 or 16: the shared A staged in LDS.
hipError_t launch_certify_wave(int waves, const CertArgs &a, int grid, hipStream_t s)
{
    switch (waves) {
    case 1: return launch_w<1, false>(a, grid, s);
    case 8: return launch_w<8, true>(a, grid, s);
    case 16: return launch_w<16, true>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

int certify_wave_blocks_per_cu(int waves, int lds)
{
    switch (waves) {
    case 1: return occ_w<1, false>(lds);
    case 8: return occ_w<8, true>(lds);
    case 16: return occ_w<16, true>(lds);
    default: return 0;
    }
}

hipError_t certify_configure(int max_lds)
{
    const void *fns[] = {(const void *)certify_kernel<64>, (const void *)certify_kernel<256>,
                         (const void *)certify_wave_kernel<1, false>, (const void *)certify_wave_kernel<8, true>,
                         (const void *)certify_wave_kernel<16, true>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lpb
