// wave_kernels.hip -- one 64-wide wavefront per LP for small tableaux.
//
// For LPs with at most 64 non-basic columns and 64*RB rows the whole solve runs
// in a single wavefront with no workgroup barrier:
//   * lane j owns column j: its non-basic variable nonb (Bland index), its
//     objective-row entry d_j and, during a pivot, its pivot-row entry prow_j;
//   * lane i (+64 r) owns row i: its basic variable, sign/sense flags, its
//     right-hand side b_i and its pivot-column entry pcol_i; the objective
//     row's right-hand side (minus the objective value) is a uniform value;
//   * the constraint columns live in LDS, column-major (lane j's column is
//     contiguous) with a column stride of an odd number of 16-byte units.
// Step 1 is a wavefront DPP/permlane reduction over the lanes' reduced costs;
// Step 2 reads the entering column (contiguous, one element per lane) and
// reduces the ratios against the row-owned right-hand sides; Step 3 sweeps each
// lane's column in 16-byte vectors, sixteen rows per group -- all reads, then
// the fma, then all writes -- with the rows' pivot-column entries broadcast
// from column e in LDS, updates the right-hand sides in the row owners'
// registers, then rewrites the swapped column and the pivot row.
// The arithmetic of every element (fma(-pcol_i, prow_j, t_ij), prow_j =
// t_lj / PE, Phase I and Phase II objective rows summed in row order) is the
// same as in the workgroup kernel, so both give bitwise-identical results.
//
// An LP whose tableau does not fit (too many surplus columns after sign
// normalisation, or too many rows) is appended to the deferred list, which the
// workgroup kernel drains in a following launch.
#include <math.h>

#include "device_common.h"
#include "internal.h"

namespace lpb {
namespace {

// Column stride (in elements) of the column-major LDS tableau: the smallest
// odd multiple of 16 bytes that holds m rows.  Lane j's column is contiguous,
// so the row sweep moves 16 bytes per lane per access, and an odd number of
// 16-byte units between neighbouring lanes' columns keeps those accesses free
// of bank conflicts.
template <typename T>
__host__ __device__ constexpr int col_stride(int m)
{
    constexpr int R = 16 / int(sizeof(T));
    const int u = (m + R - 1) / R;
    return R * (u | 1);
}

// Uniform value of row i from a per-row register array (row i lives in lane i % 64
// of block i / 64).
template <int RB, typename V>
__device__ __forceinline__ V row_get(const V (&arr)[RB], int i)
{
    if constexpr (RB == 1) {
        return lane_get(arr[0], i & 63);
    } else {
        V out = lane_get(arr[0], i & 63);
#pragma unroll
        for (int r = 1; r < RB; ++r)
            if ((i >> 6) == r) out = lane_get(arr[r], i & 63);
        return out;
    }
}

template <typename T, int RB>
struct WaveLP {
    int m, n, N, C, ldm, nart;
    int64_t k, ro, co;
    const double *A, *b, *c;
    T *tab;  // column-major: element (i, j) at tab[j * ldm + i], columns 0 .. N-1
    int rowf[RB], basis[RB];
    T pcol[RB];
    T rhs[RB];  // right-hand side of row lane + 64 r
    T z;        // right-hand side of the objective row (uniform)
    int nonb;   // this lane's column
    T d;        // this lane's objective-row entry
    int iters, it1, degp, cap;
};

// Rows of one 16-byte vector of this lane's column: v[r] = fma(-w[r], prow,
// v[r]) with w the same rows of the pivot column.
template <typename T, typename V>
__device__ __forceinline__ void update_vec(V &v, const V &w, T prow)
{
    constexpr int R = 16 / int(sizeof(T));
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = fma(-w[r], prow, v[r]);
}

// Step 3, register part: the scaled pivot row (returned; lane j's entry
// prow_j = t_lj / PE, 1 / PE in column e), the objective row and every
// right-hand side updated in their owners' registers, and the index arrays
// swapped.  P.pcol must hold the pivot column (0 for dead and padding rows).
// rowv: lane j's entry t_lj of the pivot row in the current tableau.
template <typename T, int RB>
__device__ __forceinline__ T pivot_head(WaveLP<T, RB> &P, int l, int e, T rowv)
{
    const int lane = threadIdx.x;
    const int m = P.m, C = P.C;
    const T pe = row_get<RB>(P.pcol, l);
    T prow = T(0);
    if (lane < C) prow = (lane == e) ? T(1) / pe : rowv / pe;
    const T de = lane_get(P.d, e);
    if (lane < C) P.d = fma(-de, prow, (lane == e) ? T(0) : P.d);
    // Right-hand sides: the objective row's (uniform) and every row's, in the
    // row owners' registers (dead and padding rows carry pcol 0 and stay).
    const T prow_rhs = row_get<RB>(P.rhs, l) / pe;
    P.z = fma(-de, prow_rhs, P.z);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int i = lane + 64 * r;
        if (i < m) P.rhs[r] = (i == l) ? prow_rhs : fma(-P.pcol[r], prow_rhs, P.rhs[r]);
    }
    const int bl = row_get<RB>(P.basis, l);
    const int ne = lane_get(P.nonb, e);
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (lane + 64 * r == l) P.basis[r] = ne;
    if (lane == e) P.nonb = bl;
    return prow;
}

// Step 3, LDS part: sweep this lane's column in 16-byte vectors, G vectors
// (16 rows) per group.  The same rows of the pivot column are read from
// column e by every lane (one broadcast address per load); lane e rewrites
// column e in the same sweep, but only rows whose pivot-column values every
// lane has already read, since a wavefront's LDS accesses complete in program
// order.  The pivot row and the swapped column are rewritten afterwards;
// padding rows past m take whatever values and are never read back.
template <typename T, int RB>
__device__ __forceinline__ void pivot_sweep(WaveLP<T, RB> &P, int l, int e, T prow)
{
    using V = T __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int R = 16 / int(sizeof(T));
    constexpr int G = 16 / R;  // vectors per group of 16 rows
    const int lane = threadIdx.x;
    const int m = P.m, C = P.C, ldm = P.ldm;
    T *tab = P.tab;
    if (lane < C) {
        V *col = reinterpret_cast<V *>(tab + lane * ldm);
        const V *pc = reinterpret_cast<const V *>(tab + e * ldm);
        const int nv = (m + R - 1) / R;
        int k0 = 0;
        for (; k0 + G <= nv; k0 += G) {
            V v[G], w[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                v[g] = col[k0 + g];
                w[g] = pc[k0 + g];
            }
#pragma unroll
            for (int g = 0; g < G; ++g) update_vec<T, V>(v[g], w[g], prow);
#pragma unroll
            for (int g = 0; g < G; ++g) col[k0 + g] = v[g];
        }
        for (; k0 < nv; ++k0) {
            V v = col[k0];
            const V w = pc[k0];
            update_vec<T, V>(v, w, prow);
            col[k0] = v;
        }
    }
    const T pre = lane_get(prow, e);  // 1 / PE
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int i = lane + 64 * r;
        if (i < m) tab[e * ldm + i] = (i == l) ? pre : fma(-P.pcol[r], pre, T(0));
    }
    if (lane < C) tab[lane * ldm + l] = prow;
}

template <typename T, int RB>
__device__ __forceinline__ void pivot(WaveLP<T, RB> &P, int l, int e)
{
    const int lane = threadIdx.x;
    const T rowv = (lane < P.C) ? P.tab[lane * P.ldm + l] : T(0);
    const T prow = pivot_head<T, RB>(P, l, e, rowv);
    pivot_sweep<T, RB>(P, l, e, prow);
}

// Two consecutive pivots in one sweep of the columns: (l1, e1), whose row
// vector is prow1 and column P.pcol1 (row owners), then (l2, e2) of the
// tableau the first leaves, with row vector prow2 and column pcol2.  Both
// pivots' register parts are done.  Every entry is read once, takes the
// first pivot's update and then the second's, and is written once; the
// second pivot column's entries t'_ie2 = fma(-t_ie1, prow1_e2, t_ie2) are
// formed from both columns' broadcast reads exactly as the first sweep would
// have written them.  Rows l1 and l2 and columns e1 and e2, which the two
// pivots replace rather than update, are rewritten afterwards with the
// values two separate pivots leave there, so the result is the same bit for
// bit.
template <typename T, int RB>
__device__ __forceinline__ void pivot_sweep2(WaveLP<T, RB> &P, int l1, int e1, T prow1, const T (&pcol1)[RB],
                                             int l2, int e2, T prow2)
{
    using V = T __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int R = 16 / int(sizeof(T));
    constexpr int G = 8 / R;  // vectors per group of 8 rows
    const int lane = threadIdx.x;
    const int m = P.m, C = P.C, ldm = P.ldm;
    T *tab = P.tab;
    const T p1e2 = lane_get(prow1, e2);
    if (lane < C) {
        V *col = reinterpret_cast<V *>(tab + lane * ldm);
        const V *pc1 = reinterpret_cast<const V *>(tab + e1 * ldm);
        const V *pc2 = reinterpret_cast<const V *>(tab + e2 * ldm);
        const int nv = (m + R - 1) / R;
        int k0 = 0;
        for (; k0 + G <= nv; k0 += G) {
            V v[G], w1[G], w2[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                v[g] = col[k0 + g];
                w1[g] = pc1[k0 + g];
                w2[g] = pc2[k0 + g];
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const T f2 = fma(-w1[g][q], p1e2, w2[g][q]);
                    v[g][q] = fma(-f2, prow2, fma(-w1[g][q], prow1, v[g][q]));
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) col[k0 + g] = v[g];
        }
        for (; k0 < nv; ++k0) {
            V v = col[k0];
            const V w1 = pc1[k0], w2 = pc2[k0];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const T f2 = fma(-w1[q], p1e2, w2[q]);
                v[q] = fma(-f2, prow2, fma(-w1[q], prow1, v[q]));
            }
            col[k0] = v;
        }
    }
    // Columns e1 and e2 (row owners), then rows l1 and l2 (column owners).
    const T pre1 = lane_get(prow1, e1), p2e1 = lane_get(prow2, e1), pre2 = lane_get(prow2, e2);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int i = lane + 64 * r;
        if (i < m) {
            const T c1 = (i == l1) ? pre1 : fma(-pcol1[r], pre1, T(0));
            tab[e1 * ldm + i] = (i == l2) ? p2e1 : fma(-P.pcol[r], p2e1, c1);
            tab[e2 * ldm + i] = (i == l2) ? pre2 : fma(-P.pcol[r], pre2, T(0));
        }
    }
    if (lane < C && lane != e1 && lane != e2) {
        if (l1 != l2) tab[lane * ldm + l1] = fma(-row_get<RB>(P.pcol, l1), prow2, prow1);
        tab[lane * ldm + l2] = prow2;
    }
}

// Loads column e into the per-row pivot-column registers (0 for dropped rows).
template <typename T, int RB>
__device__ __forceinline__ void load_pcol(WaveLP<T, RB> &P, int e)
{
    const int lane = threadIdx.x;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int i = lane + 64 * r;
        T a = T(0);
        if (i < P.m) a = P.tab[e * P.ldm + i];
        P.pcol[r] = (P.rowf[r] & (kRowDead | kRowPad)) ? T(0) : a;
    }
}

// Step 1: the entering column (wavefront-uniform), or -1 when none is eligible.
// Dantzig: the largest d_j, ties to the smallest Bland index; Bland: the
// smallest eligible Bland index.
template <typename T>
__device__ __forceinline__ int price(bool elig, T d, int nonb, bool bland)
{
    const int lane = threadIdx.x;
    const uint64_t any = __ballot(elig);
    if (!any) return -1;
    if (!bland) {
        const T best = wave_max_f(elig ? d : -t_inf<T>());
        const uint64_t tied = __ballot(elig && d == best);
        if (__popcll(tied) == 1) return __builtin_ctzll(tied);
        const bool in = (tied >> lane) & 1;
        const int bmin = wave_min_i(in ? nonb : kBig);
        return __builtin_ctzll(__ballot(in && nonb == bmin));
    }
    const int bmin = wave_min_i(elig ? nonb : kBig);
    return __builtin_ctzll(__ballot(elig && nonb == bmin));
}

// PAIR: look one pivot ahead and sweep two pivots at once when it finds one
// (off in the repair instantiation, whose few pivots do not pay for the
// registers).
template <typename T, int RB, bool PAIR = true>
__device__ __forceinline__ int simplex(WaveLP<T, RB> &P, T eps_opt, const SolveParams &prm, int *enter)
{
    const int lane = threadIdx.x;
    const int m = P.m, N = P.N, ldm = P.ldm, nm = P.n + P.m;
    const T tol_piv = T(prm.tol_piv);
    T *tab = P.tab;
    int deg_run = 0;
    for (;;) {
        if (P.iters >= P.cap) return kIterLimit;
        const bool bland = prm.k_deg > 0 && deg_run >= prm.k_deg;
        // Step 1.
        const bool elig = lane < N && P.d > eps_opt && P.nonb < nm;
        int e;
        if (prm.pricing == 1 && !bland) {
            // Steepest edge: each eligible lane sums the squares of its own
            // column over the live rows (contiguous in LDS).
            const uint64_t dead0 = __ballot((P.rowf[0] & (kRowDead | kRowPad)) != 0);
            const uint64_t dead1 = RB > 1 ? __ballot((P.rowf[RB - 1] & (kRowDead | kRowPad)) != 0) : 0;
            // 16-byte vectors down the column (padding rows past m are
            // masked like dead ones), one partial sum per vector component.
            using V = T __attribute__((ext_vector_type(16 / sizeof(T))));
            constexpr int R = 16 / int(sizeof(T));
            T acc[R];
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] = T(0);
            if (elig) {
                const V *col = reinterpret_cast<const V *>(tab + lane * ldm);
#pragma unroll 2
                for (int i0 = 0; i0 < m; i0 += R) {
                    const V t = col[i0 / R];
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        const int i = i0 + q;
                        const uint64_t dm = i < 64 ? dead0 : dead1;
                        acc[q] = ((dm >> (i & 63)) & 1) ? acc[q] : fma(t[q], t[q], acc[q]);
                    }
                }
            }
            T w = T(1);
#pragma unroll
            for (int q = 0; q < R; ++q) w += acc[q];
            e = price<T>(elig, elig ? P.d * P.d / w : T(0), P.nonb, false);
        } else {
            e = price<T>(elig, P.d, P.nonb, bland);
        }
        if (e < 0) return kOptimal;
        // Step 2: each lane's best row (ties to the smaller basic index), then
        // the wavefront minimum ratio, ties to the smallest basic index.
        T th_loc = t_inf<T>();
        int bb_loc = kBig, row_loc = -1;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = lane + 64 * r;
            const bool live = !(P.rowf[r] & (kRowDead | kRowPad));
            T a = T(0), bi = T(0);
            if (i < m) { a = tab[e * ldm + i]; bi = P.rhs[r]; }
            P.pcol[r] = live ? a : T(0);
            if (live && a > tol_piv) {
                const T th = (bi > T(0) ? bi : T(0)) / a;
                const int bb = P.basis[r];
                if (th < th_loc || (th == th_loc && bb < bb_loc)) { th_loc = th; bb_loc = bb; row_loc = i; }
            }
        }
        if (!__ballot(row_loc >= 0)) { *enter = lane_get(P.nonb, e); return kUnbounded; }
        const T best = wave_min_f(th_loc);
        const uint64_t tied = __ballot(row_loc >= 0 && th_loc == best);
        int src;
        if (__popcll(tied) == 1) {
            src = __builtin_ctzll(tied);
        } else {
            const bool in = (tied >> lane) & 1;
            const int bmin = wave_min_i(in ? bb_loc : kBig);
            src = __builtin_ctzll(__ballot(in && bb_loc == bmin));
        }
        const int l = lane_get(row_loc, src);
        if (lane_get(th_loc, src) == T(0)) { ++deg_run; ++P.degp; } else deg_run = 0;
        if (!PAIR || prm.pricing == 1 || P.iters + 1 >= P.cap) {
            pivot<T, RB>(P, l, e);
            ++P.iters;
            continue;
        }
        // Look one pivot ahead: this pivot's register part (objective row,
        // right-hand sides, indices) is all Steps 1 and 2 of the next
        // iteration need, with the one column they read formed from its
        // stored entries and this pivot's vectors.  When they find a second
        // pivot both go through one sweep of the columns (pivot_sweep2).
        T pcol1[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) pcol1[r] = P.pcol[r];
        const T prow1 = pivot_head<T, RB>(P, l, e, (lane < P.C) ? tab[lane * ldm + l] : T(0));
        const bool bland2 = prm.k_deg > 0 && deg_run >= prm.k_deg;
        // Column e now holds the variable that left; its reduced cost -d_e / PE
        // is negative, so e2 != e.
        const int e2 = price<T>(lane < N && P.d > eps_opt && P.nonb < nm, P.d, P.nonb, bland2);
        int l2 = -1;
        T th2 = T(0);
        if (e2 >= 0) {
            const T p1e2 = lane_get(prow1, e2);
            T th_loc2 = t_inf<T>();
            int bb_loc2 = kBig, row_loc2 = -1;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = lane + 64 * r;
                const bool live = !(P.rowf[r] & (kRowDead | kRowPad));
                T a = T(0), bi = T(0);
                if (i < m) {
                    a = (i == l) ? p1e2 : fma(-pcol1[r], p1e2, tab[e2 * ldm + i]);
                    bi = P.rhs[r];
                }
                P.pcol[r] = live ? a : T(0);
                if (live && a > tol_piv) {
                    const T th = (bi > T(0) ? bi : T(0)) / a;
                    const int bb = P.basis[r];
                    if (th < th_loc2 || (th == th_loc2 && bb < bb_loc2)) { th_loc2 = th; bb_loc2 = bb; row_loc2 = i; }
                }
            }
            if (__ballot(row_loc2 >= 0)) {
                const T best2 = wave_min_f(th_loc2);
                const uint64_t tied2 = __ballot(row_loc2 >= 0 && th_loc2 == best2);
                int src2;
                if (__popcll(tied2) == 1) {
                    src2 = __builtin_ctzll(tied2);
                } else {
                    const bool in = (tied2 >> lane) & 1;
                    const int bmin = wave_min_i(in ? bb_loc2 : kBig);
                    src2 = __builtin_ctzll(__ballot(in && bb_loc2 == bmin));
                }
                l2 = lane_get(row_loc2, src2);
                th2 = lane_get(th_loc2, src2);
            }
        }
        if (l2 < 0) {
            // Optimal or unbounded after this pivot: it goes alone, and the
            // next iteration reaches the same outcome.
#pragma unroll
            for (int r = 0; r < RB; ++r) P.pcol[r] = pcol1[r];
            pivot_sweep<T, RB>(P, l, e, prow1);
            ++P.iters;
            continue;
        }
        if (th2 == T(0)) { ++deg_run; ++P.degp; } else deg_run = 0;
        // Lane j's entry of row l2 in the tableau the first pivot leaves.
        T row2 = T(0);
        if (lane < P.C)
            row2 = (l2 == l) ? prow1
                             : fma(-row_get<RB>(pcol1, l2), prow1, (lane == e) ? T(0) : tab[lane * ldm + l2]);
        const T prow2 = pivot_head<T, RB>(P, l2, e2, row2);
        pivot_sweep2<T, RB>(P, l, e, prow1, pcol1, l2, e2, prow2);
        P.iters += 2;
    }
}

// Warm start from a final basis of a single-precision solve: either of a
// relaxation solved on a subset of the rows (warm_rows set: warm_m rows per
// LP, its basis at warm_basis + k * warm_m in relaxation numbering) or of the
// LP itself (warm_rows NULL: its basis at warm_basis + P.ro, LP numbering).
// All rows are <= after normalisation, so the tableau starts at the slack
// basis.  The start basis holds its basic structurals and the slacks of some
// of its rows; the other rows ("tight": slack non-basic) must lose their
// slacks.  Crash: every basic structural enters, in row order, at the tight
// row of largest |entry| in its column not yet used; the full LP's basis then
// is the start basis plus the slacks of any omitted rows.  Returns false when
// a pivot entry falls below tol_piv or the start basis is not square on its
// tight rows.
template <typename T, int RB>
__device__ bool crash(WaveLP<T, RB> &P, const SolveArgs &a, int64_t k)
{
    const int lane = threadIdx.x;
    const int n = P.n, m = P.m, ldm = P.ldm;
    const int wm = a.warm_rows ? a.warm_m : m;
    const int32_t *wb = a.warm_rows ? a.warm_basis + k * int64_t(wm) : a.warm_basis + P.ro;
    const int32_t *wr = a.warm_rows ? a.warm_rows + k * int64_t(wm) : nullptr;
    const T tol_piv = T(a.prm.tol_piv);
    uint64_t cand[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) cand[r] = 0;
    int nstruct = 0;
    // Tight rows: the start basis's rows, less those whose slack is basic.
    for (int r0 = 0; r0 < wm; r0 += 64) {
        const int r = r0 + lane;
        int q = -1, v = -1, qs = -1;
        if (r < wm) {
            q = wr ? wr[r] : r;
            v = wb[r];
            if (v >= n && v < n + wm) qs = wr ? wr[v - n] : v - n;  // the row of a basic slack
        }
        nstruct += __popcll(__ballot(r < wm && v >= 0 && v < n));
        for (int pass = 0; pass < 2; ++pass) {
            const int qq = pass == 0 ? q : qs;
            uint64_t bits = __ballot(qq >= 0 && qq < m);
            while (bits) {
                const int src = __builtin_ctzll(bits);
                bits &= bits - 1;
                const int qi = lane_get(qq, src);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    if ((qi >> 6) == rb) {
                        if (pass == 0) cand[rb] |= uint64_t(1) << (qi & 63);
                        else cand[rb] &= ~(uint64_t(1) << (qi & 63));
                    }
            }
        }
    }
    int ntight = 0;
#pragma unroll
    for (int r = 0; r < RB; ++r) ntight += __popcll(cand[r]);
    if (ntight != nstruct) return false;
    for (int r0 = 0; r0 < wm; r0 += 64) {
        const int r = r0 + lane;
        const int v = r < wm ? wb[r] : -1;
        uint64_t bits = __ballot(r < wm && v >= 0 && v < n);
        while (bits) {
            const int src = __builtin_ctzll(bits);
            bits &= bits - 1;
            const int j = lane_get(v, src);
            const uint64_t at = __ballot(P.nonb == j);
            if (!at) return false;  // listed twice
            const int c = __builtin_ctzll(at);
            T best = T(-1);
            int rl = -1;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int i = lane + 64 * rb;
                if (i < m && ((cand[rb] >> lane) & 1)) {
                    const T t = fabs(P.tab[c * ldm + i]);
                    if (t > best) { best = t; rl = i; }
                }
            }
            const T bmax = wave_max_f(best);
            if (!(bmax > tol_piv)) return false;
            const int l = lane_get(rl, __builtin_ctzll(__ballot(rl >= 0 && best == bmax)));
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                if ((l >> 6) == rb) cand[rb] &= ~(uint64_t(1) << (l & 63));
            load_pcol<T, RB>(P, c);
            pivot<T, RB>(P, l, c);
            ++P.iters;
        }
    }
    return true;
}

// Repair of a start basis from a single-precision solve (the final basis of
// an FP32 relaxation, or of the FP32 solve of the LP itself), which the FP64
// arithmetic may find slightly primal or dual infeasible.  A start that is
// dual feasible up to the single-precision level: the dual simplex method,
// with d_j taken as min(d_j, 0), restores primal feasibility -- the leaving
// row is the most negative right-hand side below -tol_p (ties to the smallest
// basic Bland index), the entering column the smallest min(d_j, 0) / t_lj over
// t_lj < -tol_piv (ties to the smallest Bland index) -- and the primal method
// then removes any d_j > eps_opt left.  A start that is primal feasible but
// not dual feasible goes straight to the primal method.  Returns the status,
// or -1 when the start is neither (the caller then solves from the slack
// basis).
template <typename T, int RB>
__device__ int dual_repair(WaveLP<T, RB> &P, T eps_opt, T tol_dual, T tol_p, const SolveParams &prm, int *enter)
{
    const int lane = threadIdx.x;
    const int m = P.m, N = P.N, ldm = P.ldm, nm = P.n + P.m;
    const T tol_piv = T(prm.tol_piv);
    if (__ballot(lane < N && P.d > tol_dual && P.nonb < nm)) {
        bool infeas = false;
#pragma unroll
        for (int r = 0; r < RB; ++r)
            infeas |= lane + 64 * r < m && !(P.rowf[r] & (kRowDead | kRowPad)) && P.rhs[r] < -tol_p;
        if (__ballot(infeas)) return -1;
        return simplex<T, RB, false>(P, eps_opt, prm, enter);
    }
    for (;;) {
        if (P.iters >= P.cap) return kIterLimit;
        T vl = t_inf<T>();
        int bl = kBig, rl = -1;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = lane + 64 * r;
            const T v = P.rhs[r];
            if (i < m && !(P.rowf[r] & (kRowDead | kRowPad)) && v < -tol_p &&
                (v < vl || (v == vl && P.basis[r] < bl))) {
                vl = v; bl = P.basis[r]; rl = i;
            }
        }
        if (!__ballot(rl >= 0)) break;  // primal feasible
        const T vmin = wave_min_f(vl);
        const uint64_t tied = __ballot(rl >= 0 && vl == vmin);
        int src = __builtin_ctzll(tied);
        if (__popcll(tied) > 1) {
            const bool in = (tied >> lane) & 1;
            const int bmin = wave_min_i(in ? bl : kBig);
            src = __builtin_ctzll(__ballot(in && bl == bmin));
        }
        const int l = lane_get(rl, src);
        T tlj = T(0);
        if (lane < N) tlj = P.tab[lane * ldm + l];
        const bool el = lane < N && P.nonb < nm && tlj < -tol_piv;
        if (!__ballot(el)) return kInfeasible;  // row l cannot reach its bound
        const T ratio = el ? (P.d < T(0) ? P.d : T(0)) / tlj : t_inf<T>();
        const T rmin = wave_min_f(ratio);
        const uint64_t rt = __ballot(el && ratio == rmin);
        int e = __builtin_ctzll(rt);
        if (__popcll(rt) > 1) {
            const bool in = (rt >> lane) & 1;
            const int bmin = wave_min_i(in ? P.nonb : kBig);
            e = __builtin_ctzll(__ballot(in && P.nonb == bmin));
        }
        load_pcol<T, RB>(P, e);
        pivot<T, RB>(P, l, e);
        ++P.iters;
    }
    return simplex<T, RB, false>(P, eps_opt, prm, enter);
}

// Bytes of LDS the wave kernel keeps in front of the tableau: the surplus
// column -> row map and the row -> constraint map of a screened LP.  (The
// objective c stays in registers and is fetched across lanes with
// ds_bpermute; x is staged in the tableau's first columns once the pivots are
// done.)  Keeping this small lets one more 50 x 50 FP64 LP fit per CU.
__host__ __device__ constexpr int64_t wave_aux_bytes(int rb, bool gather)
{
    return align16(4 * 64 * rb) + (gather ? align16(4 * 64 * rb) : 0);
}

// Doubles of A each lane prefetches: LPs with m * n <= 64 * NPF have their
// whole constraint matrix loaded into registers one LP ahead.  Batches of
// larger (or row-gathered) LPs use the instantiation without the prefetch
// registers, which leaves room for more wavefronts per SIMD.
constexpr int NPF = 40;

// An LP's geometry and input data, loaded into registers ahead of its solve.
template <int RB, int PFD>
struct Fetch {
    int64_t k, ro, co;
    int m, n;
    const double *A;
    bool has_a;
    double av[PFD > 0 ? PFD : 1];  // A in flat row-major order, element lane + 64 t
    double bv[RB];   // b of row lane + 64 r
    int sv[RB];      // sense of row lane + 64 r
    int rid[RB];     // constraint of the shared LP that row lane + 64 r is (shared only)
    bool bad_row;    // a row index outside the shared LP (this lane's rows)
    double cv;       // c of column lane
};

// Issues the loads of work item `item`.  The LP's geometry is wavefront-uniform
// (computed, or read and broadcast for batches of mixed sizes); every data
// load is an unconditional buffer load through a uniform descriptor whose
// range check returns 0 past the LP's end, so no branch separates the loads and
// nothing waits for them before their first use in the next LP's setup.
template <int RB, int PFD>
__device__ __forceinline__ void fetch(const SolveArgs &a, int64_t item, Fetch<RB, PFD> &F)
{
    const int lane = threadIdx.x;
    const int64_t k = a.ids ? int64_t(uniform(a.ids[item])) : item;
    F.k = k;
    int m, n;
    int64_t aoff;
    if (a.um > 0) {
        m = a.um; n = a.un;
        aoff = k * int64_t(m) * n;
        F.ro = k * m;
        F.co = k * n;
    } else {
        // All five loads in flight before the first broadcast waits for them.
        const int mk = a.m[k], nk = a.n[k];
        const int64_t ak = a.aoff[k], rk = a.roff[k], ck = a.coff[k];
        m = uniform(mk); n = uniform(nk);
        aoff = uniform64(ak);
        F.ro = uniform64(rk);
        F.co = uniform64(ck);
    }
    F.m = m; F.n = n;
    F.A = a.shared ? a.A : a.A + aoff;
    F.bad_row = false;
    if (a.shared) {
        // One LP's constraints shared by the batch; a screened LP takes the
        // rows its subset names (gathered, so A is read row by row later).
        const int32_t *sub = a.row_subset ? a.row_subset + k * int64_t(m) : nullptr;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = lane + 64 * r;
            int q = i;
            if (sub && i < m) q = sub[i];
            const bool okq = q >= 0 && q < a.m_full;
            F.bad_row |= i < m && !okq;
            q = okq ? q : 0;
            F.rid[r] = q;
            F.bv[r] = (i < m) ? a.b[q] : 0.0;
            F.sv[r] = (i < m) ? int(a.sense[q]) : 0;
        }
    } else {
        const __amdgpu_buffer_rsrc_t rb = buffer_over(a.b + F.ro, m * int(sizeof(double)));
        const __amdgpu_buffer_rsrc_t rsn = buffer_over(a.sense + F.ro, m);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = lane + 64 * r;
            F.rid[r] = i;
            F.bv[r] = buffer_f64(rb, i * int(sizeof(double)));
            F.sv[r] = int(int8_t(__builtin_amdgcn_raw_buffer_load_b8(rsn, i, 0, 0)));
        }
    }
    F.cv = buffer_f64(buffer_over(a.c + F.co, n * int(sizeof(double))), lane * int(sizeof(double)));
    const int mn = m * n;
    F.has_a = PFD > 0 && mn <= 64 * PFD && !(a.shared && a.row_subset);
    if constexpr (PFD > 0) if (F.has_a) {
        const __amdgpu_buffer_rsrc_t rs = buffer_over(F.A, mn * int(sizeof(double)));
#pragma unroll
        for (int t = 0; t < PFD; ++t) F.av[t] = buffer_f64(rs, (lane + 64 * t) * int(sizeof(double)));
    }
}

template <typename T, int RB, int PFD, bool WARM = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(PFD > 0 ? 2 : (sizeof(T) == 4 ? (RB == 1 ? 5 : 4) : 3)))) void simplex_wave_kernel(SolveArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x;
    int *colrow = reinterpret_cast<int *>(smem);
    int *rowid = reinterpret_cast<int *>(smem + align16(4 * 64 * RB));
    const int64_t aux = wave_aux_bytes(RB, a.shared && a.row_subset);
    const int64_t total = a.num_dev ? int64_t(a.id_base) + *a.num_dev : a.num;
    // Work items: blockIdx.x and blockIdx.x + G first, then 2G + the queue
    // counter; the next item is always known one LP ahead, so its data can be
    // in flight while the current LP pivots.
    const int64_t G = gridDim.x;
    int64_t cur = blockIdx.x, nxt = blockIdx.x + G;
    Fetch<RB, PFD> F;
    if (cur < total) fetch<RB, PFD>(a, cur, F);
    while (cur < total) {
        // The queue counter is read here and used only when this LP is done.
        // (An increment with wrap at 2^32 - 1 is a plain +1 here; unlike an add
        // it is not rewritten into a wavefront-combined atomic whose result is
        // broadcast, and waited for, right away.)
        int qv = 0;
        if (lane == 0) qv = int(atomicInc(reinterpret_cast<unsigned *>(a.queue), 0xffffffffu));
        const int64_t k = F.k;
        WaveLP<T, RB> P;
        P.k = k;
        P.m = F.m; P.n = F.n;
        P.A = F.A;
        P.ro = F.ro;
        P.co = F.co;
        const int m = P.m, n = P.n;

        // A1: sign-normalise and classify rows; surplus columns by ballot.
        bool bad = F.bad_row;
        const bool gather = a.shared && a.row_subset;
        if (gather) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
                if (lane + 64 * r < m) rowid[lane + 64 * r] = F.rid[r];
        }
        double bv[RB];
        int sc[RB];
        int ng = 0, nart = 0, neq = 0;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = lane + 64 * r;
            int f = kRowPad;
            const double bi = F.bv[r];
            if (i < m) {
                const int s = F.sv[r];
                bad |= !isfinite(bi) || s < kLE || s > kEQ;
                const bool neg = bi < 0.0;
                int sen = (s < kLE || s > kEQ) ? kLE : s;
                if (neg && sen != kEQ) sen = (sen == kLE) ? kGE : kLE;
                f = (neg ? kRowNeg : 0) | (sen << 1);
            }
            bv[r] = bi;
            P.rowf[r] = f;
            P.rhs[r] = (i < m) ? T((f & kRowNeg) ? -bi : bi) : T(0);
            const int sen = (f >> 1) & 3;
            const uint64_t ge = __ballot(i < m && sen == kGE);
            const uint64_t ar = __ballot(i < m && sen != kLE);
            const uint64_t eq = __ballot(i < m && sen == kEQ);
            sc[r] = -1;
            if (i < m && sen == kGE) {
                const int g = ng + __popcll(ge & lanemask_lt(lane));
                sc[r] = n + g;
                if (g < 64 * RB) colrow[g] = i;
            }
            ng += __popcll(ge);
            nart += __popcll(ar);
            neq += __popcll(eq);
        }
        P.N = n + ng;
        P.C = P.N;
        P.ldm = col_stride<T>(m);
        P.nart = nart;
        const int64_t need = aux + int64_t(P.C) * P.ldm * int64_t(sizeof(T));
        const bool fits = P.C <= 64 && m <= 64 * RB && need <= a.lds_bytes;
        if (!fits && lane == 0) {
            const int slot = a.defer_base + atomicAdd(a.defer_count, 1);
            a.defer_ids[slot] = int32_t(k);
        }
        const int N = P.N, C = P.C, ldm = P.ldm;
        T *tab = reinterpret_cast<T *>(smem + aux);
        P.tab = tab;

        // A2: index arrays and the tableau (column-major in LDS).
        P.nonb = kBig;
        const double cj = fresh_copy(F.cv);
        if (fits) {
        if (lane < n) {
            P.nonb = lane;
            bad |= !isfinite(cj);
        } else if (lane < N) {
            P.nonb = n + colrow[lane - n];
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = lane + 64 * r;
            P.basis[r] = (((P.rowf[r] >> 1) & 3) == kLE) ? n + i : n + m + i;
        }
        {
            // A scattered from flat row-major order into the columns.  Element
            // f = lane + 64 t sits at row f / n, column f % n; stepping t by one
            // advances the column by 64 % n and the row by 64 / n, plus one
            // when the column wraps.
            const int mn = m * n;
            const int dq = 64 / n, dr = 64 - dq * n;
            int ri = lane / n, cj2 = lane - (lane / n) * n;
            if (PFD > 0 && F.has_a) {
                // The element's position cj2 * ldm + ri advances by
                // dr * ldm + dq per step, and by 1 - n * ldm more when the
                // column wraps; only the last, partial step needs a bounds test.
                // (Prefetched elements past m * n read as 0, so every register
                // can be checked for finiteness.)
                const int full = mn >> 6;
                const int step = dr * ldm + dq, wrap = 1 - n * ldm;
                int pos = cj2 * ldm + ri;
#pragma unroll
                for (int t = 0; t < (PFD > 0 ? PFD : 1); ++t) bad |= !isfinite(F.av[t]);
#pragma unroll
                for (int t = 0; t < (PFD > 0 ? PFD : 1); ++t) {
                    if (t < full || (t == full && lane + 64 * t < mn)) tab[pos] = T(F.av[t]);
                    cj2 += dr;
                    pos += step;
                    if (cj2 >= n) { cj2 -= n; pos += wrap; }
                }
            } else {
                // (Eight loads in flight for FP32 LPs of up to 64 rows keeps them
                // within the registers of five wavefronts per SIMD.)
                constexpr int UB = (sizeof(T) == 4 && RB == 1) ? 8 : 16;
                for (int f0 = 0; f0 < mn; f0 += 64 * UB) {
                    double av[UB];
                    if (gather) {
                        // Row f / n of the LP is constraint rowid[f / n] of the shared LP.
                        int rr = ri, cc = cj2;
#pragma unroll
                        for (int u = 0; u < UB; ++u) {
                            const int f = f0 + 64 * u + lane;
                            av[u] = 0.0;
                            if (f < mn) av[u] = P.A[int64_t(rowid[rr < m ? rr : m - 1]) * n + cc];
                            rr += dq;
                            cc += dr;
                            if (cc >= n) { cc -= n; ++rr; }
                        }
                    } else {
#pragma unroll
                        for (int u = 0; u < UB; ++u) {
                            const int f = f0 + 64 * u + lane;
                            av[u] = (f < mn) ? P.A[f] : 0.0;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < UB; ++u) {
                        if (f0 + 64 * u + lane < mn) {
                            bad |= !isfinite(av[u]);
                            tab[cj2 * ldm + ri] = T(av[u]);
                        }
                        ri += dq;
                        cj2 += dr;
                        if (cj2 >= n) { cj2 -= n; ++ri; }
                    }
                }
            }
            // Rows with b < 0 are negated (sign normalisation).
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                uint64_t neg = __ballot(lane + 64 * r < m && (P.rowf[r] & kRowNeg));
                while (neg) {
                    const int i = 64 * r + __builtin_ctzll(neg);
                    neg &= neg - 1;
                    if (lane < n) tab[lane * ldm + i] = -tab[lane * ldm + i];
                }
            }
            // Surplus columns, one row per lane.
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = lane + 64 * r;
                if (i < m)
                    for (int g = 0; g < ng; ++g) tab[(n + g) * ldm + i] = (sc[r] == n + g) ? T(-1) : T(0);
            }
        }
        }  // fits
        const double cnorm = wave_max_f(fabs(cj));
        double bm = 0.0;
#pragma unroll
        for (int r = 0; r < RB; ++r) bm = fmax(bm, fabs(bv[r]));
        const double bnorm = wave_max_f(bm);
        // The registers of F are free again: start loading the next LP.  (The
        // last LP of a wavefront reloads itself, so the loads are unconditional
        // and land in the registers the current LP's came in.)
        fetch<RB, PFD>(a, nxt < total ? nxt : cur, F);
        if (!fits) {
            cur = nxt;
            nxt = 2 * G + lane_get(qv, 0);
            continue;
        }
        const bool invalid = __ballot(bad) != 0;
        P.iters = 0; P.it1 = 0; P.degp = 0;
        P.cap = a.prm.max_iters > 0 ? a.prm.max_iters : 50 * (m + n + (m - neq) + nart);
        P.d = T(0);
        P.z = T(0);
        int status = kOptimal, enter = -1;

        // Warm start (repair instantiation): only from a relaxation that ended
        // optimal (its status is still in status[k]) with few violated rows,
        // and only for all-<= LPs; any other LP is solved from the slack basis
        // right here.  An LP whose repair fails is deferred.
        bool warm_ok = false, warm_defer = false;
        if (invalid) {
            status = kInvalid;
        } else {
            if constexpr (WARM) {
                warm_ok = nart == 0 && a.status[k] == kOptimal &&
                          !(a.warm_viol && a.warm_viol[k] > a.warm_max_viol);
                if (warm_ok) warm_defer = !crash<T, RB>(P, a, k);
            }
            if (warm_defer) {
                // nothing more here: the LP goes to the solve from the slack basis
            } else if (nart > 0) {
                // Phase I objective row: sum of the artificial rows in row order.
                T acc = T(0), zacc = T(0);
                for (int i = 0; i < m; ++i) {
                    const int sen = (row_get<RB>(P.rowf, i) >> 1) & 3;
                    if (sen != kLE) {
                        if (lane < C) acc += tab[lane * ldm + i];
                        zacc += row_get<RB>(P.rhs, i);
                    }
                }
                P.d = acc;
                P.z = zacc;
                const double dmax = wave_max_f(lane < N ? fabs(double(acc)) : 0.0);
                const double dscale = fmax(1.0, dmax);
                const int r = simplex<T, RB, !WARM>(P, T(a.prm.tol_opt * dscale), a.prm, &enter);
                P.it1 = P.iters;
                enter = -1;
                if (r == kIterLimit) status = kIterLimit;
                else if (r == kUnbounded) status = kNumerical;
                else {
                    const double wstar = -double(P.z);
                    if (wstar < -a.prm.tol_feas * (1.0 + bnorm)) status = kInfeasible;
                }
                if (status == kOptimal) {
                    // Drive basic artificials out in row order; drop redundant rows.
                    const T tol_piv = T(a.prm.tol_piv);
#pragma unroll
                    for (int r = 0; r < RB; ++r) {
                        uint64_t am = __ballot(lane + 64 * r < m && P.basis[r] >= n + m);
                        while (am) {
                            const int bit = __builtin_ctzll(am);
                            am &= am - 1;
                            const int i = 64 * r + bit;
                            bool ok = false;
                            if (lane < N && P.nonb < n + m) ok = fabs(tab[lane * ldm + i]) > tol_piv;
                            const int e = price<T>(ok, T(0), P.nonb, true);
                            if (e >= 0) {
                                load_pcol<T, RB>(P, e);
                                pivot<T, RB>(P, i, e);
                            } else if (lane == bit) {
                                P.rowf[r] |= kRowDead;
                            }
                        }
                    }
                }
            }
            if (status == kOptimal && !warm_defer) {
                // Phase II objective row: c priced out over the basis, rows in order.
                T cb[RB];
                uint64_t nz[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int bvr = P.basis[r];
                    const double cbv = __shfl(cj, bvr < n ? bvr : 0);  // c of the row's basic variable
                    cb[r] = (!(P.rowf[r] & (kRowDead | kRowPad)) && bvr < n) ? T(cbv) : T(0);
                    nz[r] = __ballot(cb[r] != T(0));
                }
                const double cnb = __shfl(cj, (P.nonb >= 0 && P.nonb < n) ? P.nonb : 0);
                T acc = (lane < N && P.nonb < n) ? T(cnb) : T(0), zacc = T(0);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    uint64_t mk = nz[r];
                    while (mk) {
                        const int bit = __builtin_ctzll(mk);
                        mk &= mk - 1;
                        const T f = lane_get(cb[r], bit);
                        if (lane < C) acc = fma(-f, tab[lane * ldm + 64 * r + bit], acc);
                        zacc = fma(-f, lane_get(P.rhs[r], bit), zacc);
                    }
                }
                P.d = acc;
                P.z = zacc;
                if (WARM && warm_ok) {
                    // Single-precision level for the start's reduced costs.
                    status = dual_repair<T, RB>(P, T(a.prm.tol_opt * fmax(1.0, cnorm)), T(1e-5 * fmax(1.0, cnorm)),
                                                T(a.prm.tol_feas * (1.0 + bnorm)), a.prm, &enter);
                    warm_defer = status != kOptimal;
                } else {
                    status = simplex<T, RB, !WARM>(P, T(a.prm.tol_opt * fmax(1.0, cnorm)), a.prm, &enter);
                }
            }
        }
        if (WARM && warm_defer) {
            if (lane == 0) {
                // Not optimal any more: the workgroup kernel that drains the
                // deferred list then solves it from the slack basis.
                a.status[k] = kNumerical;
                const int slot = a.defer_base + atomicAdd(a.defer_count, 1);
                a.defer_ids[slot] = int32_t(k);
            }
            cur = nxt;
            nxt = 2 * G + lane_get(qv, 0);
            continue;
        }

        // A8: extraction through an LDS staging vector.
        // The tableau's first columns are free now (the rhs column N is read
        // below and lies past them): x is staged there.
        T *xv = tab;
        if (lane < n) xv[lane] = T(0);
        if (status == kOptimal) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = lane + 64 * r;
                const int bvr = P.basis[r];
                if (i < m && bvr < n && !(P.rowf[r] & kRowDead)) xv[bvr] = P.rhs[r];
            }
        }
        const double xj = (lane < n) ? double(xv[lane]) : 0.0;
        if (lane < n) a.x[P.co + lane] = (status == kOptimal) ? xj : __builtin_nan("");
        double z = (lane < n) ? fma(cj, xj, 0.0) : 0.0;
        int nbs = (lane < n && xj != 0.0) ? 1 : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            z += __shfl_xor(z, off);
            nbs += __shfl_xor(nbs, off);
        }
        if (lane == 0) {
            double objv = z;
            if (status == kUnbounded) objv = __builtin_inf();
            else if (status != kOptimal) objv = __builtin_nan("");
            a.obj[k] = objv;
            a.status[k] = status;
            if (a.enter_out) a.enter_out[k] = (status == kUnbounded) ? enter : -1;
            if (a.stats) {
                int32_t *st = a.stats + 8 * k;
                if (a.refine_stats) {
                    st[3] = warm_ok ? 2 : 1;  // 2: started from the relaxation's basis
                    st[4] = P.iters;
                } else {
                    st[0] = P.it1;
                    st[1] = P.iters - P.it1;
                    st[2] = P.degp;
                    st[3] = 0;
                    st[4] = 0;
                    st[5] = 0;
                }
                st[6] = 1;
                st[7] = nbs;
            }
        }
        if (a.basis_out) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = lane + 64 * r;
                if (i < m) a.basis_out[P.ro + i] = (P.rowf[r] & kRowDead) ? -1 : P.basis[r];
            }
        }
        cur = nxt;
        nxt = 2 * G + lane_get(qv, 0);
    }
    if (lane == 0) finish_launch(a.queue, a.done, a.reset_extra);
}


template <typename T, int RB, int PFD, bool WARM = false>
hipError_t launch_t(const SolveArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((simplex_wave_kernel<T, RB, PFD, WARM>), dim3(grid), dim3(64), a.lds_bytes, s, a);
    return hipGetLastError();
}

template <typename T, int RB, int PFD, bool WARM = false>
int occ_t(int lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &blocks, (const void *)simplex_wave_kernel<T, RB, PFD, WARM>, 64, lds) != hipSuccess)
        return 0;
    return blocks;
}

template <typename T>
hipError_t launch_rb(int rb, bool pf, const SolveArgs &a, int grid, hipStream_t s)
{
    if (rb == 1) return pf ? launch_t<T, 1, NPF>(a, grid, s) : launch_t<T, 1, 0>(a, grid, s);
    if (rb == 2) return pf ? launch_t<T, 2, NPF>(a, grid, s) : launch_t<T, 2, 0>(a, grid, s);
    return hipErrorInvalidValue;
}

template <typename T>
int occ_rb(int rb, bool pf, int lds)
{
    if (rb == 1) return pf ? occ_t<T, 1, NPF>(lds) : occ_t<T, 1, 0>(lds);
    if (rb == 2) return pf ? occ_t<T, 2, NPF>(lds) : occ_t<T, 2, 0>(lds);
    return 0;
}

}  // namespace

int64_t wave_lds_aux_bytes(int rb, bool gather) { return wave_aux_bytes(rb, gather); }

int64_t wave_tab_bytes(int m, int cols, bool fp32)
{
    return fp32 ? int64_t(cols) * col_stride<float>(m) * 4 : int64_t(cols) * col_stride<double>(m) * 8;
}

int wave_prefetch_elems() { return 64 * NPF; }

hipError_t launch_simplex_wave(bool fp32, int rb, bool pf, const SolveArgs &a, int grid, hipStream_t s)
{
    return fp32 ? launch_rb<float>(rb, pf, a, grid, s) : launch_rb<double>(rb, pf, a, grid, s);
}

int simplex_wave_blocks_per_cu(bool fp32, int rb, bool pf, int lds)
{
    return fp32 ? occ_rb<float>(rb, pf, lds) : occ_rb<double>(rb, pf, lds);
}

hipError_t launch_simplex_wave_warm(int rb, const SolveArgs &a, int grid, hipStream_t s)
{
    if (!a.warm_basis || (a.warm_rows && a.warm_m < 1)) return hipErrorInvalidValue;
    if (rb == 1) return launch_t<double, 1, 0, true>(a, grid, s);
    if (rb == 2) return launch_t<double, 2, 0, true>(a, grid, s);
    return hipErrorInvalidValue;
}

int simplex_wave_warm_blocks_per_cu(int rb, int lds)
{
    if (rb == 1) return occ_t<double, 1, 0, true>(lds);
    if (rb == 2) return occ_t<double, 2, 0, true>(lds);
    return 0;
}

hipError_t simplex_wave_configure(int max_lds)
{
    const void *fns[] = {(const void *)simplex_wave_kernel<float, 1, NPF>, (const void *)simplex_wave_kernel<double, 1, NPF>,
                         (const void *)simplex_wave_kernel<float, 2, NPF>, (const void *)simplex_wave_kernel<double, 2, NPF>,
                         (const void *)simplex_wave_kernel<float, 1, 0>,   (const void *)simplex_wave_kernel<double, 1, 0>,
                         (const void *)simplex_wave_kernel<float, 2, 0>,   (const void *)simplex_wave_kernel<double, 2, 0>,
                         (const void *)simplex_wave_kernel<double, 1, 0, true>,
                         (const void *)simplex_wave_kernel<double, 2, 0, true>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lpb
