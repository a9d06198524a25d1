// simplex_kernels.hip -- the batched dense-tableau simplex for gfx950.
//
// One workgroup solves one LP at a time and pops the next LP from a work
// counter (a persistent launch sized to what the device holds at once).  The
// paper maps one CUDA block to one LP (Sec. 5.1, load balancing) and uses the
// block's threads inside the tableau; here a workgroup of NT threads (one or
// more 64-wide wavefronts) does the same, with the tableau kept in LDS when it
// fits the launch's LDS budget and in an HBM scratch slot of the workgroup
// otherwise.
//
// The tableau is the condensed ("exchange") form of the paper's Sec. 4.1
// tableau: the m basic columns are unit vectors and are not stored, so a row
// holds the N non-basic columns and the right-hand side, and a pivot swaps the
// entering and leaving variables' columns in place.  Rows 0..m-1 are the
// constraints, row m the objective: reduced costs d_j (entering candidates
// have d_j > 0) and, in the rhs cell, minus the current objective value.
// basis[i] / nonb[j] hold the Bland index of the variable of row i / column j.
//
// Per iteration (Sec. 4.1):
//   Step 1 (pricing): argmax of d_j > eps_opt over eligible columns, ties to
//     the smallest Bland index; Bland's smallest-index rule after k_deg
//     consecutive degenerate pivots, until a pivot makes progress.
//   Step 2 (ratio): argmin of max(b_i, 0) / a_ie over rows with a_ie > tol_piv,
//     ties to the smallest Bland index of the basic variable; none: unbounded.
//     Wavefront DPP reductions and ballots on (key, Bland index), then one
//     slot per wavefront in LDS, stand in for the paper's Data[]/Indices[]
//     arrays, with +inf as the "MAX" sentinel.
//   Step 3 (pivot): pivot row / PE; every other row (objective included) minus
//     a_ie times the new pivot row (Listing 1); the entering column becomes the
//     leaving variable's column: 1/PE in the pivot row, -a_ie/PE elsewhere.
//     Every element is rewritten with one fma, the same expression wherever
//     the tableau lives, so results do not depend on the placement or the
//     workgroup size.  Up to three consecutive pivots whose Steps 1-2 can be
//     taken from the earlier pivots' vectors share one sweep (each element
//     takes their rules in order, so results are those of separate sweeps).
// Phase I (Sec. 4) maximises -(sum of artificials) when some row needs one;
// basic artificials at zero are driven out and redundant rows dropped, then
// Phase II prices c out over the basis and continues.
#include <math.h>

#include "device_common.h"
#include "internal.h"

namespace lpb {
namespace {

constexpr int LE = 0, GE = 1, EQ = 2;
constexpr int ST_OPTIMAL = 0, ST_INFEASIBLE = 1, ST_UNBOUNDED = 2, ST_ITER = 3,
              ST_NUMERICAL = 4, ST_INVALID = 5;
constexpr int BIG = 0x7fffffff;
constexpr int ROW_NEG = 1, ROW_DEAD = 8;

template <typename T>
struct Ctrl {
    int ng, nart, neq, bad;
    int next;
    int cnt;  // scratch tally (warm start)
    int pad[2];
    double bnorm, cnorm;
    T rv[16];
    int ri[16];
    int rp[16];
    double rd[16];
};

__device__ __forceinline__ int row_sense(int f) { return (f >> 1) & 3; }

// ---- reductions ------------------------------------------------------------

template <typename T, int NT>
__device__ __forceinline__ void block_argmin(T &k1, int &k2, int &p, Ctrl<T> *sh)
{
    wave_argmin_dpp(k1, k2, p);
    if constexpr (NT > 64) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) { sh->rv[w] = k1; sh->ri[w] = k2; sh->rp[w] = p; }
        __syncthreads();
        k1 = sh->rv[0]; k2 = sh->ri[0]; p = sh->rp[0];
#pragma unroll
        for (int q = 1; q < NT / 64; ++q) {
            T o1 = sh->rv[q];
            int o2 = sh->ri[q];
            if (o1 < k1 || (o1 == k1 && o2 < k2)) { k1 = o1; k2 = o2; p = sh->rp[q]; }
        }
        __syncthreads();
    }
}

template <typename T, int NT>
__device__ __forceinline__ double block_max(double v, Ctrl<T> *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
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

// ---- one LP ------------------------------------------------------------------

template <typename T, int NT>
struct LP {
    // geometry
    int m, n, N, C, ld, nart;
    int64_t k, ro, co;
    const double *A, *b, *c;
    const int32_t *rows;  // screened LP: row i is constraint rows[i] of the shared LP
    int m_full;
    // Constraint of the (shared) LP that row i reads, clamped into range.
    __device__ __forceinline__ int row_of(int i) const
    {
        if (!rows) return i;
        const int q = rows[i];
        return (q >= 0 && q < m_full) ? q : 0;
    }
    // LDS arrays
    Ctrl<T> *sh;
    int *basis, *nonb, *rowf, *colrow;
    T *pcol, *prow;    // pivot column and (scaled) pivot row of a pivot
    T *pcol2, *prow2;  // the same for the second pivot of a fused pair
    T *pcol3, *prow3;  // and for the third of a fused triple
    T *tab;  // LDS or HBM
    // counters (uniform across the workgroup)
    int iters, it1, degp, cap;
};

// Step 3's vectors for a pivot on (l, e) of the current tableau: the scaled
// pivot row prow_j = t_lj / PE (1 / PE in column e) and the pivot column
// pcol_i = t_ie (0 for dropped rows; row m is the objective row).  No barrier.
template <typename T, int NT>
__device__ __forceinline__ void pivot_vectors(LP<T, NT> &P, int l, int e, bool have_col = false)
{
    const int tid = threadIdx.x;
    const T *tab = P.tab;
    const int ld = P.ld, C = P.C, m = P.m;
    const T pe = tab[(int64_t)l * ld + e];
    for (int j = tid; j < C; j += NT)
        P.prow[j] = (j == e) ? T(1) / pe : tab[(int64_t)l * ld + j] / pe;
    // have_col: Step 2 already stored rows 0..m-1 of the column (same thread
    // per row), so only the objective row's entry is read here.
    if (have_col) {
        if (tid == 0) P.pcol[m] = tab[(int64_t)m * ld + e];
    } else {
        for (int i = tid; i <= m; i += NT)
            P.pcol[i] = (i < m && (P.rowf[i] & ROW_DEAD)) ? T(0) : tab[(int64_t)i * ld + e];
    }
}

// Step 3's sweep: every tableau entry t_ij becomes fma(-pcol_i, prow_j, t_ij)
// -- with 0 in place of t_ij in the pivot column e, and prow_j itself in the
// pivot row l -- for the pivot whose vectors are in P.prow / P.pcol; with
// PAIR, the result then takes the second pivot's rule the same way (vectors
// in P.prow2 / P.pcol2, row l2, column e2).  Lanes move 16 bytes (R entries)
// per access, U accesses in flight -- all loads, then the fmas, then all
// stores.  Rows start 16-byte aligned (tableau_ld); the entries past C up to
// the row stride are padding, updated with whatever they hold and never read
// back (the pivot-row buffers are padded the same way).
//   * Wide rows (more than 64 U / 2 vectors): each wavefront takes whole rows.
//   * Narrow rows: each wavefront takes RW = 64 U / nv rows at a time, its
//     lanes spread over those rows' vectors (item q = lane + 64 u is vector
//     q % nv of row q / nv), so a narrow tableau still keeps every lane busy
//     and many accesses in flight -- with a tableau in device memory the
//     sweep is bound by the accesses in flight, not by the bytes.
// No barrier.
template <typename T, int NT, int NP>
__device__ __forceinline__ void sweep_impl(LP<T, NT> &P, int l1, int e1, int l2, int e2, int l3, int e3)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int W = NT / 64;
    T *tab = P.tab;
    const int ld = P.ld, C = P.C, m = P.m;
    using V = T __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int R = 16 / int(sizeof(T));
    constexpr int U = 4;
    const int nv = (C + R - 1) / R;
    const V *pr1 = reinterpret_cast<const V *>(P.prow);
    const V *pr2 = reinterpret_cast<const V *>(P.prow2);
    const V *pr3 = reinterpret_cast<const V *>(P.prow3);
    // One entry's update: the first pivot's rule, then the second's and the
    // third's (NP pivots).
    auto upd = [&](int i, int j, T v, T w1, T f1, T w2, T f2, T w3, T f3) {
        T t = (i == l1) ? w1 : fma(-f1, w1, (j == e1) ? T(0) : v);
        if constexpr (NP >= 2) t = (i == l2) ? w2 : fma(-f2, w2, (j == e2) ? T(0) : t);
        if constexpr (NP >= 3) t = (i == l3) ? w3 : fma(-f3, w3, (j == e3) ? T(0) : t);
        return t;
    };
    const int rw = (64 * U) / nv;  // rows per wavefront step on the narrow path
    if (rw < 2) {
        for (int i = wave; i <= m; i += W) {
            V *row = reinterpret_cast<V *>(tab + (int64_t)i * ld);
            const T f1 = P.pcol[i];
            const T f2 = NP >= 2 ? P.pcol2[i] : T(0);
            const T f3 = NP >= 3 ? P.pcol3[i] : T(0);
            for (int k0 = lane; k0 < nv; k0 += 64 * U) {
                V v[U], w1[U], w2[U], w3[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int k = k0 + 64 * u;
                    if (k < nv) {
                        v[u] = row[k];
                        w1[u] = pr1[k];
                        if constexpr (NP >= 2) w2[u] = pr2[k];
                        if constexpr (NP >= 3) w3[u] = pr3[k];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int k = k0 + 64 * u;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        v[u][r] = upd(i, k * R + r, v[u][r], w1[u][r], f1, NP >= 2 ? w2[u][r] : T(0), f2,
                                      NP >= 3 ? w3[u][r] : T(0), f3);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int k = k0 + 64 * u;
                    if (k < nv) row[k] = v[u];
                }
            }
        }
        return;
    }
    // Narrow rows: this lane's items, as (row offset, vector) pairs.
    int ro[U], kv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int q = lane + 64 * u;
        ro[u] = q / nv;
        kv[u] = q - ro[u] * nv;
        if (ro[u] >= rw) ro[u] = m + 1;  // past the last row: no item
    }
    for (int i0 = wave * rw; i0 <= m; i0 += W * rw) {
        V v[U], w1[U], w2[U], w3[U];
        T f1[U], f2[U], f3[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + ro[u];
            if (i <= m) {
                v[u] = reinterpret_cast<const V *>(tab + (int64_t)i * ld)[kv[u]];
                w1[u] = pr1[kv[u]];
                f1[u] = P.pcol[i];
                if constexpr (NP >= 2) {
                    w2[u] = pr2[kv[u]];
                    f2[u] = P.pcol2[i];
                }
                if constexpr (NP >= 3) {
                    w3[u] = pr3[kv[u]];
                    f3[u] = P.pcol3[i];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + ro[u];
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[u][r] = upd(i, kv[u] * R + r, v[u][r], w1[u][r], f1[u], NP >= 2 ? w2[u][r] : T(0),
                              NP >= 2 ? f2[u] : T(0), NP >= 3 ? w3[u][r] : T(0), NP >= 3 ? f3[u] : T(0));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + ro[u];
            if (i <= m) reinterpret_cast<V *>(tab + (int64_t)i * ld)[kv[u]] = v[u];
        }
    }
}

template <typename T, int NT>
__device__ __forceinline__ void sweep1(LP<T, NT> &P, int l, int e)
{
    sweep_impl<T, NT, 1>(P, l, e, -1, -1, -1, -1);
}

// Step 3: pivot on (l, e).  Every thread takes part; ends with a barrier.
template <typename T, int NT>
__device__ __forceinline__ void pivot(LP<T, NT> &P, int l, int e)
{
    pivot_vectors<T, NT>(P, l, e);
    __syncthreads();
    sweep1<T, NT>(P, l, e);
    if (threadIdx.x == 0) {
        const int t = P.basis[l];
        P.basis[l] = P.nonb[e];
        P.nonb[e] = t;
    }
    __syncthreads();
}

// Two consecutive pivots, (l1, e1) and then (l2, e2) of the tableau that the
// first leaves, in ONE pass over the tableau: every entry is read once,
// updated by the first pivot's rule and then by the second's -- the same
// operations in the same order as two separate sweeps, so the result is the
// same bit for bit -- and written once, which halves the tableau traffic of
// the pair.  P.prow / P.pcol hold the first pivot's vectors, P.prow2 / P.pcol2
// the second's (computed from the first's without the tableau being swept).
// No barrier.
template <typename T, int NT>
__device__ __forceinline__ void sweep2(LP<T, NT> &P, int l1, int e1, int l2, int e2)
{
    sweep_impl<T, NT, 2>(P, l1, e1, l2, e2, -1, -1);
}

// Three consecutive pivots in one pass (vectors in P.prow3 / P.pcol3 for the
// third), the same operations in the same order as three sweeps.  No barrier.
template <typename T, int NT>
__device__ __forceinline__ void sweep3(LP<T, NT> &P, int l1, int e1, int l2, int e2, int l3, int e3)
{
    sweep_impl<T, NT, 3>(P, l1, e1, l2, e2, l3, e3);
}

// Steps 1-3 until a halt condition.  Returns ST_OPTIMAL, ST_UNBOUNDED or ST_ITER;
// *enter receives the entering Bland index when unbounded.
template <typename T, int NT>
__device__ __forceinline__ int simplex(LP<T, NT> &P, T eps_opt, const SolveParams &prm, int *enter)
{
    const int tid = threadIdx.x;
    const int m = P.m, N = P.N, C = P.C, ld = P.ld, nm = P.n + P.m;
    const T tol_piv = T(prm.tol_piv);
    T *tab = P.tab;
    int deg_run = 0;
    for (;;) {
        if (P.iters >= P.cap) return ST_ITER;
        const bool bland = prm.k_deg > 0 && deg_run >= prm.k_deg;
        // Step 1: entering column.
        T k1 = t_inf<T>();
        int k2 = BIG, p = -1;
        const T *obj = tab + (int64_t)m * ld;
        const bool steep = prm.pricing == 1 && !bland;
        for (int j = tid; j < N; j += NT) {
            const T d = obj[j];
            const int bj = P.nonb[j];
            if (d > eps_opt && bj < nm) {
                T key = bland ? T(0) : -d;
                if (steep) {
                    // Steepest edge: d_j^2 / (1 + sum of column j's squares
                    // over the live rows); threads walk down their columns,
                    // rows i summed into partial sum i mod R, the partial sums
                    // then added in order -- the wavefront kernel's order, so
                    // both kernels choose the same column.
                    constexpr int R = 16 / int(sizeof(T));
                    T acc[R];
#pragma unroll
                    for (int q = 0; q < R; ++q) acc[q] = T(0);
                    for (int i0 = 0; i0 < m; i0 += R) {
#pragma unroll
                        for (int q = 0; q < R; ++q) {
                            const int i = i0 + q;
                            if (i < m && !(P.rowf[i] & ROW_DEAD)) {
                                const T t = tab[(int64_t)i * ld + j];
                                acc[q] = fma(t, t, acc[q]);
                            }
                        }
                    }
                    T w = T(1);
#pragma unroll
                    for (int q = 0; q < R; ++q) w += acc[q];
                    key = -(d * d / w);
                }
                if (key < k1 || (key == k1 && bj < k2)) { k1 = key; k2 = bj; p = j; }
            }
        }
        block_argmin<T, NT>(k1, k2, p, P.sh);
        if (p < 0) return ST_OPTIMAL;
        const int e = p;
        // Step 2: leaving row.
        k1 = t_inf<T>(); k2 = BIG; p = -1;
        const bool keep_col = prm.pricing != 1 && P.iters + 1 < P.cap;  // the look-ahead path reuses it
        for (int i = tid; i < m; i += NT) {
            if (P.rowf[i] & ROW_DEAD) {
                if (keep_col) P.pcol[i] = T(0);
                continue;
            }
            const T a = tab[(int64_t)i * ld + e];
            if (keep_col) P.pcol[i] = a;
            if (a > tol_piv) {
                const T bi = tab[(int64_t)i * ld + N];
                const T th = (bi > T(0) ? bi : T(0)) / a;
                const int bb = P.basis[i];
                if (th < k1 || (th == k1 && bb < k2)) { k1 = th; k2 = bb; p = i; }
            }
        }
        block_argmin<T, NT>(k1, k2, p, P.sh);
        if (p < 0) { *enter = P.nonb[e]; return ST_UNBOUNDED; }
        if (k1 == T(0)) { ++deg_run; ++P.degp; } else deg_run = 0;
        const int l = p;
        if (prm.pricing == 1 || P.iters + 1 >= P.cap) {
            pivot<T, NT>(P, l, e);
            ++P.iters;
            continue;
        }
        // Look one pivot ahead.  The tableau the pivot on (l, e) leaves is
        // t'_ij = fma(-pcol_i, prow_j, t_ij) (0 for t_ij in column e; prow_j
        // in row l), so Steps 1 and 2 of the next iteration need only the
        // objective row, one column and the right-hand sides of it, computed
        // here from the pivot's vectors without sweeping the tableau.  When
        // they find a second pivot both go through one sweep (sweep2), or,
        // when a third is found the same way, all three (sweep3).
        pivot_vectors<T, NT>(P, l, e, true);
        if (tid == 0) {
            const int t = P.basis[l];
            P.basis[l] = P.nonb[e];
            P.nonb[e] = t;
        }
        __syncthreads();
        // Step 1 of the next iteration (column e now holds the variable that
        // left; its reduced cost -d_e / PE is negative, so e2 != e).
        const bool bland2 = prm.k_deg > 0 && deg_run >= prm.k_deg;
        const T fm = P.pcol[m];
        k1 = t_inf<T>(); k2 = BIG; p = -1;
        for (int j = tid; j < N; j += NT) {
            const T d = fma(-fm, P.prow[j], (j == e) ? T(0) : obj[j]);
            const int bj = P.nonb[j];
            if (d > eps_opt && bj < nm) {
                const T key = bland2 ? T(0) : -d;
                if (key < k1 || (key == k1 && bj < k2)) { k1 = key; k2 = bj; p = j; }
            }
        }
        block_argmin<T, NT>(k1, k2, p, P.sh);
        const int e2 = p;
        int l2 = -1;
        if (e2 >= 0) {
            // Step 2 of the next iteration.
            k1 = t_inf<T>(); k2 = BIG; p = -1;
            const T pc2 = P.prow[e2], prhs = P.prow[N];
            for (int i = tid; i < m; i += NT) {
                if (P.rowf[i] & ROW_DEAD) {
                    P.pcol2[i] = T(0);
                    continue;
                }
                const T a = (i == l) ? pc2 : fma(-P.pcol[i], pc2, tab[(int64_t)i * ld + e2]);
                P.pcol2[i] = a;  // the second pivot's column, if this step finds a row
                if (a > tol_piv) {
                    const T bi = (i == l) ? prhs : fma(-P.pcol[i], prhs, tab[(int64_t)i * ld + N]);
                    const T th = (bi > T(0) ? bi : T(0)) / a;
                    const int bb = P.basis[i];
                    if (th < k1 || (th == k1 && bb < k2)) { k1 = th; k2 = bb; p = i; }
                }
            }
            block_argmin<T, NT>(k1, k2, p, P.sh);
            l2 = p;
        }
        if (l2 < 0) {
            // Optimal or unbounded after this pivot: it goes alone, and the
            // next iteration reaches the same outcome.
            sweep1<T, NT>(P, l, e);
            __syncthreads();
            ++P.iters;
            continue;
        }
        if (k1 == T(0)) { ++deg_run; ++P.degp; } else deg_run = 0;
        // The second pivot's vectors, entry by entry as pivot_vectors would
        // compute them from the swept tableau.
        {
            const T pc2 = P.prow[e2];
            const T pe2 = (l2 == l) ? pc2 : fma(-P.pcol[l2], pc2, tab[(int64_t)l2 * ld + e2]);
            const T f2 = P.pcol[l2];
            for (int j = tid; j < C; j += NT) {
                const T t = (l2 == l) ? P.prow[j]
                                      : fma(-f2, P.prow[j], (j == e) ? T(0) : tab[(int64_t)l2 * ld + j]);
                P.prow2[j] = (j == e2) ? T(1) / pe2 : t / pe2;
            }
            // Rows 0..m-1 of the column were stored by Step 2 above.
            if (tid == 0) {
                const int i = m;
                P.pcol2[i] = fma(-P.pcol[i], pc2, tab[(int64_t)i * ld + e2]);
                const int t = P.basis[l2];
                P.basis[l2] = P.nonb[e2];
                P.nonb[e2] = t;
            }
        }
        __syncthreads();
        // Look a third pivot ahead the same way, from both pivots' vectors:
        // entry (i, j) after the two pivots is
        //   t'_ij  = (i == l ) ? prow_j  : fma(-pcol_i,  prow_j,  j == e  ? 0 : t_ij)
        //   t''_ij = (i == l2) ? prow2_j : fma(-pcol2_i, prow2_j, j == e2 ? 0 : t'_ij).
        int e3 = -1, l3 = -1;
        if (P.iters + 2 < P.cap) {
            const bool bland3 = prm.k_deg > 0 && deg_run >= prm.k_deg;
            const T fm2 = P.pcol2[m];
            k1 = t_inf<T>(); k2 = BIG; p = -1;
            for (int j = tid; j < N; j += NT) {
                const T d1 = fma(-fm, P.prow[j], (j == e) ? T(0) : obj[j]);
                const T d = fma(-fm2, P.prow2[j], (j == e2) ? T(0) : d1);
                const int bj = P.nonb[j];
                if (d > eps_opt && bj < nm) {
                    const T key = bland3 ? T(0) : -d;
                    if (key < k1 || (key == k1 && bj < k2)) { k1 = key; k2 = bj; p = j; }
                }
            }
            block_argmin<T, NT>(k1, k2, p, P.sh);
            e3 = p;
            if (e3 >= 0) {
                k1 = t_inf<T>(); k2 = BIG; p = -1;
                const T pc1 = P.prow[e3], pc2b = P.prow2[e3], prhs1 = P.prow[N], prhs2 = P.prow2[N];
                for (int i = tid; i < m; i += NT) {
                    if (P.rowf[i] & ROW_DEAD) {
                        P.pcol3[i] = T(0);
                        continue;
                    }
                    const T a1 = (i == l) ? pc1 : fma(-P.pcol[i], pc1, (e3 == e) ? T(0) : tab[(int64_t)i * ld + e3]);
                    const T a = (i == l2) ? pc2b : fma(-P.pcol2[i], pc2b, (e3 == e2) ? T(0) : a1);
                    P.pcol3[i] = a;
                    if (a > tol_piv) {
                        const T b1 = (i == l) ? prhs1 : fma(-P.pcol[i], prhs1, tab[(int64_t)i * ld + N]);
                        const T bi = (i == l2) ? prhs2 : fma(-P.pcol2[i], prhs2, b1);
                        const T th = (bi > T(0) ? bi : T(0)) / a;
                        const int bb = P.basis[i];
                        if (th < k1 || (th == k1 && bb < k2)) { k1 = th; k2 = bb; p = i; }
                    }
                }
                block_argmin<T, NT>(k1, k2, p, P.sh);
                l3 = p;
            }
        }
        if (l3 < 0) {
            sweep2<T, NT>(P, l, e, l2, e2);
            __syncthreads();
            P.iters += 2;
            continue;
        }
        if (k1 == T(0)) { ++deg_run; ++P.degp; } else deg_run = 0;
        // The third pivot's vectors.
        {
            const T pe3 = P.pcol3[l3];
            for (int j = tid; j < C; j += NT) {
                const T t1 = (l3 == l) ? P.prow[j]
                                       : fma(-P.pcol[l3], P.prow[j], (j == e) ? T(0) : tab[(int64_t)l3 * ld + j]);
                const T t = (l3 == l2) ? P.prow2[j] : fma(-P.pcol2[l3], P.prow2[j], (j == e2) ? T(0) : t1);
                P.prow3[j] = (j == e3) ? T(1) / pe3 : t / pe3;
            }
            if (tid == 0) {
                const int i = m;
                const T a1 = fma(-P.pcol[i], P.prow[e3], (e3 == e) ? T(0) : tab[(int64_t)i * ld + e3]);
                P.pcol3[i] = fma(-P.pcol2[i], P.prow2[e3], (e3 == e2) ? T(0) : a1);
                const int t = P.basis[l3];
                P.basis[l3] = P.nonb[e3];
                P.nonb[e3] = t;
            }
        }
        __syncthreads();
        sweep3<T, NT>(P, l, e, l2, e2, l3, e3);
        __syncthreads();
        P.iters += 3;
    }
}

// A1/A2: non-basic and basic index arrays, then the tableau rows
// (sign-normalised so every rhs is >= 0, with a -1 surplus entry per >= row).
// Returns whether this thread saw a non-finite entry of A or b.
template <typename T, int NT>
__device__ __forceinline__ bool fill_tableau(LP<T, NT> &P)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int W = NT / 64;
    const int m = P.m, n = P.n, N = P.N, C = P.C, ld = P.ld;
    T *tab = P.tab;
    for (int j = tid; j < N; j += NT) P.nonb[j] = (j < n) ? j : n + P.colrow[j - n];
    for (int i = tid; i < m; i += NT)
        P.basis[i] = (row_sense(P.rowf[i]) == LE) ? n + i : n + m + i;
    bool bad = false;
    for (int i = wave; i < m; i += W) {
        const double sg = (P.rowf[i] & ROW_NEG) ? -1.0 : 1.0;
        const double *Ai = P.A + (int64_t)P.row_of(i) * n;
        T *row = tab + (int64_t)i * ld;
        for (int j = lane; j < C; j += 64) {
            double v;
            if (j < n) {
                const double aij = Ai[j];
                bad |= !isfinite(aij);
                v = sg * aij;
            } else if (j < N) {
                v = (P.colrow[j - n] == i) ? -1.0 : 0.0;
            } else {
                v = sg * P.b[P.row_of(i)];
            }
            row[j] = T(v);
        }
    }
    return bad;
}

// Phase II objective row: c priced out over the current basis, rows in order.
template <typename T, int NT>
__device__ __forceinline__ void price_out(LP<T, NT> &P)
{
    const int tid = threadIdx.x;
    const int m = P.m, n = P.n, N = P.N, C = P.C, ld = P.ld;
    T *tab = P.tab;
    for (int i = tid; i < m; i += NT) {
        const int bv = P.basis[i];
        P.pcol[i] = ((P.rowf[i] & ROW_DEAD) || bv >= n) ? T(0) : T(P.c[bv]);
    }
    __syncthreads();
    for (int j = tid; j < C; j += NT) {
        const int bj = (j < N) ? P.nonb[j] : BIG;
        T acc = (bj < n) ? T(P.c[bj]) : T(0);
        for (int i = 0; i < m; ++i) {
            const T cb = P.pcol[i];
            if (cb != T(0)) acc = fma(-cb, tab[(int64_t)i * ld + j], acc);
        }
        tab[(int64_t)m * ld + j] = acc;
    }
    __syncthreads();
}

// Warm start of an FP64 re-solve from the final basis of the single-precision
// solve of the same LP (basis at warm_basis + P.ro, LP numbering; all rows <=
// after normalisation, so the tableau starts at the slack basis).  Tight rows
// are those whose slack is non-basic in the start basis; every basic
// structural enters, in row order, at the tight row of largest |entry| in its
// column not yet used (ties to the lower row).  Returns false -- the tableau
// then holds some mix and must be rebuilt -- when the start basis is not square
// on its tight rows or a pivot entry falls below tol_piv.  P.colrow (unused
// without surplus columns) holds the tight-row flags.
template <typename T, int NT>
__device__ __forceinline__ bool crash(LP<T, NT> &P, const SolveArgs &a)
{
    const int tid = threadIdx.x;
    const int m = P.m, n = P.n, N = P.N, ld = P.ld;
    const T *tab = P.tab;
    const int32_t *wb = a.warm_basis + P.ro;
    Ctrl<T> *sh = P.sh;
    int *tight = P.colrow;
    for (int i = tid; i < m; i += NT) tight[i] = 1;
    if (tid == 0) { sh->bad = 0; sh->cnt = 0; }
    __syncthreads();
    int cnt = 0;  // basic structurals minus tight rows, this thread's share
    for (int r = tid; r < m; r += NT) {
        const int v = wb[r];
        if (v < 0 || v >= n + m) sh->bad = 1;  // not a basis of this all-<= LP
        else if (v >= n) tight[v - n] = 0;     // basic slack: its row is not tight
        else ++cnt;
    }
    __syncthreads();
    for (int i = tid; i < m; i += NT) cnt -= tight[i];
    if (cnt) atomicAdd(&sh->cnt, cnt);
    __syncthreads();
    if (sh->bad || sh->cnt != 0) return false;
    const T tol_piv = T(a.prm.tol_piv);
    for (int r = 0; r < m; ++r) {
        const int v = wb[r];
        if (v >= n) continue;
        // The structural's column (it must still be non-basic).
        T k1 = T(0);
        int k2 = BIG, p = -1;
        for (int j = tid; j < N; j += NT)
            if (P.nonb[j] == v) { k2 = j; p = j; }
        block_argmin<T, NT>(k1, k2, p, sh);
        if (p < 0) return false;
        const int c = p;
        // The unused tight row of largest |entry| (ties to the lower row).
        k1 = t_inf<T>(); k2 = BIG; p = -1;
        for (int i = tid; i < m; i += NT) {
            if (!tight[i]) continue;
            const T t = -fabs(tab[(int64_t)i * ld + c]);
            if (t < k1 || (t == k1 && i < k2)) { k1 = t; k2 = i; p = i; }
        }
        block_argmin<T, NT>(k1, k2, p, sh);
        if (p < 0 || !(-k1 > tol_piv)) return false;
        if (tid == 0) tight[p] = 0;
        pivot<T, NT>(P, p, c);
        ++P.iters;
    }
    return true;
}

// Repair of the crashed start (objective row priced out): the dual simplex
// method, with d_j taken as min(d_j, 0), restores primal feasibility when the
// start is dual feasible up to the single-precision level tol_dual -- leaving
// row: the most negative right-hand side below -tol_p (ties to the smallest
// basic Bland index); entering column: the smallest min(d_j, 0) / t_lj over
// t_lj < -tol_piv (ties to the smallest Bland index) -- then the primal method
// removes any d_j > eps_opt left.  A primal feasible start that is not dual
// feasible goes straight to the primal method.  Returns the status, or -1
// when the start is neither.
template <typename T, int NT>
__device__ __forceinline__ int dual_repair(LP<T, NT> &P, T eps_opt, T tol_dual, T tol_p, const SolveParams &prm, int *enter)
{
    const int tid = threadIdx.x;
    const int m = P.m, N = P.N, ld = P.ld, nm = P.n + P.m;
    T *tab = P.tab;
    const T tol_piv = T(prm.tol_piv);
    Ctrl<T> *sh = P.sh;
    // Dual and primal feasibility of the start.
    double dmax = -1.0, pinf = -1.0;
    for (int j = tid; j < N; j += NT)
        if (P.nonb[j] < nm && tab[(int64_t)m * ld + j] > tol_dual) dmax = 1.0;
    for (int i = tid; i < m; i += NT)
        if (!(P.rowf[i] & ROW_DEAD) && tab[(int64_t)i * ld + N] < -tol_p) pinf = 1.0;
    const bool dual_bad = block_max<T, NT>(dmax, sh) > 0.0;
    const bool primal_bad = block_max<T, NT>(pinf, sh) > 0.0;
    if (dual_bad) return primal_bad ? -1 : simplex<T, NT>(P, eps_opt, prm, enter);
    for (;;) {
        if (P.iters >= P.cap) return ST_ITER;
        T k1 = t_inf<T>();
        int k2 = BIG, p = -1;
        for (int i = tid; i < m; i += NT) {
            if (P.rowf[i] & ROW_DEAD) continue;
            const T v = tab[(int64_t)i * ld + N];
            const int bb = P.basis[i];
            if (v < -tol_p && (v < k1 || (v == k1 && bb < k2))) { k1 = v; k2 = bb; p = i; }
        }
        block_argmin<T, NT>(k1, k2, p, sh);
        if (p < 0) break;  // primal feasible
        const int l = p;
        k1 = t_inf<T>(); k2 = BIG; p = -1;
        for (int j = tid; j < N; j += NT) {
            const int bj = P.nonb[j];
            const T t = tab[(int64_t)l * ld + j];
            if (bj < nm && t < -tol_piv) {
                const T d = tab[(int64_t)m * ld + j];
                const T ratio = (d < T(0) ? d : T(0)) / t;
                if (ratio < k1 || (ratio == k1 && bj < k2)) { k1 = ratio; k2 = bj; p = j; }
            }
        }
        block_argmin<T, NT>(k1, k2, p, sh);
        if (p < 0) return ST_INFEASIBLE;  // row l cannot reach its bound
        pivot<T, NT>(P, l, p);
        ++P.iters;
    }
    return simplex<T, NT>(P, eps_opt, prm, enter);
}

// Solve LP k with the tableau at P.tab (LDS or HBM).  Row classification
// (rowf, colrow, Ctrl counts) has been done by the caller.
template <typename T, int NT>
__device__ __forceinline__ void solve_lp(LP<T, NT> &P, const SolveArgs &a, int placement)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int W = NT / 64;
    const int m = P.m, n = P.n, N = P.N, C = P.C, ld = P.ld;
    Ctrl<T> *sh = P.sh;
    T *tab = P.tab;

    bool bad = fill_tableau<T, NT>(P);
    double cmax = 0.0;
    for (int j = tid; j < n; j += NT) {
        const double cj = P.c[j];
        bad |= !isfinite(cj);
        cmax = fmax(cmax, fabs(cj));
    }
    if (bad) sh->bad = 1;
    double bmax = 0.0;
    for (int i = tid; i < m; i += NT) bmax = fmax(bmax, fabs(P.b[P.row_of(i)]));
    __syncthreads();
    const double cnorm = block_max<T, NT>(cmax, sh);
    const double bnorm = block_max<T, NT>(bmax, sh);
    int status = ST_OPTIMAL, enter = -1;
    const bool invalid = sh->bad != 0;
    P.iters = 0; P.it1 = 0; P.degp = 0;
    P.cap = a.prm.max_iters > 0 ? a.prm.max_iters
                                : 50 * (m + n + (m - sh->neq) + P.nart);

    // Warm start of an FP64 re-solve from the single-precision solve's final
    // basis of this LP (not for screened solves, whose repair the wavefront
    // kernel does): only when that solve ended optimal -- its status is still
    // in status[k] -- with few violated rows, and only for all-<= LPs.
    bool warm = !invalid && a.warm_basis && !a.warm_rows && P.nart == 0 && a.status[P.k] == ST_OPTIMAL &&
                !(a.warm_viol && a.warm_viol[P.k] > a.warm_max_viol);
    if (warm && !crash<T, NT>(P, a)) {
        // The crash stopped part-way: rebuild the slack-basis tableau.
        warm = false;
        __syncthreads();
        fill_tableau<T, NT>(P);
        P.iters = 0;
        __syncthreads();
    }
    if (invalid) {
        status = ST_INVALID;
    } else {
        if (P.nart > 0) {
            // Phase I objective row: the sum of the artificial rows (in row order).
            double dmax = 0.0;
            for (int j = tid; j < C; j += NT) {
                T acc = T(0);
                for (int i = 0; i < m; ++i)
                    if (row_sense(P.rowf[i]) != LE) acc += tab[(int64_t)i * ld + j];
                tab[(int64_t)m * ld + j] = acc;
                if (j < N) dmax = fmax(dmax, fabs(double(acc)));
            }
            __syncthreads();
            const double dscale = fmax(1.0, block_max<T, NT>(dmax, sh));
            const int r = simplex<T, NT>(P, T(a.prm.tol_opt * dscale), a.prm, &enter);
            P.it1 = P.iters;
            enter = -1;
            if (r == ST_ITER) status = ST_ITER;
            else if (r == ST_UNBOUNDED) status = ST_NUMERICAL;
            else {
                const double wstar = -double(tab[(int64_t)m * ld + N]);
                if (wstar < -a.prm.tol_feas * (1.0 + bnorm)) status = ST_INFEASIBLE;
            }
            if (status == ST_OPTIMAL) {
                // Drive basic artificials out, in row order; drop redundant rows.
                const T tol_piv = T(a.prm.tol_piv);
                for (int i = 0; i < m; ++i) {
                    if (P.basis[i] < n + m) continue;
                    T k1 = T(0);
                    int k2 = BIG, p = -1;
                    for (int j = tid; j < N; j += NT) {
                        const int bj = P.nonb[j];
                        if (bj < n + m && fabs(tab[(int64_t)i * ld + j]) > tol_piv && bj < k2) {
                            k2 = bj; p = j;
                        }
                    }
                    block_argmin<T, NT>(k1, k2, p, sh);
                    if (p >= 0) {
                        pivot<T, NT>(P, i, p);
                    } else {
                        if (tid == 0) P.rowf[i] |= ROW_DEAD;
                        __syncthreads();
                    }
                }
            }
        }
        if (status == ST_OPTIMAL) {
            // Phase II objective row: c priced out over the current basis.
            price_out<T, NT>(P);
            const T eps_opt = T(a.prm.tol_opt * fmax(1.0, cnorm));
            if (warm) {
                // Single-precision level for the start's reduced costs.
                status = dual_repair<T, NT>(P, eps_opt, T(1e-5 * fmax(1.0, cnorm)),
                                            T(a.prm.tol_feas * (1.0 + bnorm)), a.prm, &enter);
                if (status < 0) {
                    // Neither primal nor dual feasible: solve from the slack basis.
                    warm = false;
                    __syncthreads();
                    fill_tableau<T, NT>(P);
                    P.iters = 0;
                    __syncthreads();
                    price_out<T, NT>(P);
                    status = simplex<T, NT>(P, eps_opt, a.prm, &enter);
                }
            } else {
                status = simplex<T, NT>(P, eps_opt, a.prm, &enter);
            }
        }
    }

    // A8: extraction.  x_j = rhs of the row where j is basic, else 0;
    // objective recomputed in FP64 from the input c by wavefront 0 in a fixed order.
    T *xv = P.prow;  // reuse as an n-vector
    for (int j = tid; j < n; j += NT) xv[j] = T(0);
    __syncthreads();
    int nbs = 0;
    if (status == ST_OPTIMAL) {
        for (int i = tid; i < m; i += NT) {
            const int bv = P.basis[i];
            if (bv < n && !(P.rowf[i] & ROW_DEAD)) xv[bv] = tab[(int64_t)i * ld + N];
        }
    }
    __syncthreads();
    double *x = a.x + P.co;
    if (status == ST_OPTIMAL) {
        for (int j = tid; j < n; j += NT) x[j] = double(xv[j]);
    } else {
        for (int j = tid; j < n; j += NT) x[j] = __builtin_nan("");
    }
    if (wave == 0) {
        double z = 0.0;
        for (int j = lane; j < n; j += 64) {
            const double xj = double(xv[j]);
            z = fma(P.c[j], xj, z);
            nbs += (xj != 0.0);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            z += __shfl_xor(z, off);
            nbs += __shfl_xor(nbs, off);
        }
        if (lane == 0) {
            double objv = z;
            if (status == ST_UNBOUNDED) objv = __builtin_inf();
            else if (status != ST_OPTIMAL) objv = __builtin_nan("");
            a.obj[P.k] = objv;
            a.status[P.k] = status;
            if (a.enter_out) a.enter_out[P.k] = (status == ST_UNBOUNDED) ? enter : -1;
            if (a.stats) {
                int32_t *st = a.stats + 8 * P.k;
                if (a.refine_stats) {
                    st[3] = warm ? 2 : 1;  // 2: started from the single-precision basis
                    st[4] = P.iters;
                } else {
                    st[0] = P.it1;
                    st[1] = P.iters - P.it1;
                    st[2] = P.degp;
                    st[3] = 0;
                    st[4] = 0;
                    st[5] = 0;
                }
                st[6] = placement;
                st[7] = nbs;
            }
        }
    }
    if (a.basis_out)
        for (int i = tid; i < m; i += NT)
            a.basis_out[P.ro + i] = (P.rowf[i] & ROW_DEAD) ? -1 : P.basis[i];
    __syncthreads();
}

// An LP this launch was not planned for (its index arrays or tableau would
// not fit the launch's LDS or device-memory slot): reported NUMERICAL
// without touching the tableau storage.
template <typename T, int NT>
__device__ __forceinline__ void reject_lp(const LP<T, NT> &P, const SolveArgs &a)
{
    const int tid = threadIdx.x;
    for (int j = tid; j < P.n; j += NT) a.x[P.co + j] = __builtin_nan("");
    if (a.basis_out)
        for (int i = tid; i < P.m; i += NT) a.basis_out[P.ro + i] = -1;
    if (tid == 0) {
        a.obj[P.k] = __builtin_nan("");
        a.status[P.k] = ST_NUMERICAL;
        if (a.enter_out) a.enter_out[P.k] = -1;
        if (a.stats) {
            int32_t *st = a.stats + 8 * P.k;
            if (a.refine_stats) {
                st[3] = 1;
                st[4] = 0;
            } else {
                for (int q = 0; q < 8; ++q) st[q] = 0;
            }
        }
    }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void simplex_kernel(SolveArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    Ctrl<T> *sh = reinterpret_cast<Ctrl<T> *>(smem);
    const int64_t total = a.num_dev ? int64_t(a.id_base) + *a.num_dev : a.num;
    int64_t item = blockIdx.x;
    while (item < total) {
        if (tid == 0) sh->next = gridDim.x + atomicAdd(a.queue, 1);
        const int64_t k = a.ids ? int64_t(a.ids[item]) : item;
        LP<T, NT> P;
        P.k = k;
        if (a.um > 0) {
            P.m = a.um; P.n = a.un;
            P.A = a.A + k * int64_t(a.um) * a.un;
            P.ro = k * a.um;
            P.co = k * a.un;
        } else {
            P.m = a.m[k]; P.n = a.n[k];
            P.A = a.A + a.aoff[k];
            P.ro = a.roff[k];
            P.co = a.coff[k];
        }
        P.b = a.b + P.ro;
        P.c = a.c + P.co;
        P.rows = nullptr;
        P.m_full = P.m;
        const int8_t *sense = a.sense + P.ro;
        if (a.shared) {
            // One LP's constraints shared by the batch (optionally a row subset of them).
            P.A = a.A;
            P.b = a.b;
            sense = a.sense;
            P.m_full = a.m_full;
            P.rows = a.row_subset ? a.row_subset + k * int64_t(P.m) : nullptr;
        }
        const int m = P.m, n = P.n;
        LdsLayout L = lds_layout(m, n + m, sizeof(T), sizeof(Ctrl<T>));
        P.sh = sh;
        P.basis = reinterpret_cast<int *>(smem + L.basis);
        P.nonb = reinterpret_cast<int *>(smem + L.nonb);
        P.rowf = reinterpret_cast<int *>(smem + L.rowf);
        P.colrow = reinterpret_cast<int *>(smem + L.colrow);
        P.pcol = reinterpret_cast<T *>(smem + L.pcol);
        P.prow = reinterpret_cast<T *>(smem + L.prow);
        P.pcol2 = reinterpret_cast<T *>(smem + L.pcol2);
        P.prow2 = reinterpret_cast<T *>(smem + L.prow2);
        P.pcol3 = reinterpret_cast<T *>(smem + L.pcol3);
        P.prow3 = reinterpret_cast<T *>(smem + L.prow3);
        if (L.tab > int64_t(a.lds_bytes)) {
            reject_lp<T, NT>(P, a);
            __syncthreads();
            item = sh->next;
            __syncthreads();
            continue;
        }

        // A1: sign-normalise and classify rows (sense after flipping rows with b < 0).
        if (tid == 0) sh->bad = 0;
        __syncthreads();
        bool bad = false;
        for (int i = tid; i < m; i += NT) {
            const int q = P.row_of(i);
            const double bi = P.b[q];
            const int s = sense[q];
            bad |= !isfinite(bi) || s < LE || s > EQ;
            if (P.rows) bad |= P.rows[i] < 0 || P.rows[i] >= P.m_full;
            const bool neg = bi < 0.0;
            int sen = (s < LE || s > EQ) ? LE : s;
            if (neg && sen != EQ) sen = (sen == LE) ? GE : LE;
            P.rowf[i] = (neg ? ROW_NEG : 0) | (sen << 1);
        }
        if (bad) sh->bad = 1;
        __syncthreads();
        // Surplus columns of >= rows in row order (wavefront ballots), counts.
        if (wave == 0) {
            int ng = 0, nart = 0, neq = 0;
            for (int i0 = 0; i0 < m; i0 += 64) {
                const int i = i0 + lane;
                const int sen = (i < m) ? row_sense(P.rowf[i]) : LE;
                const uint64_t ge = __ballot(i < m && sen == GE);
                const uint64_t ar = __ballot(i < m && sen != LE);
                const uint64_t eq = __ballot(i < m && sen == EQ);
                if (i < m && sen == GE)
                    P.colrow[ng + __popcll(ge & ((uint64_t(1) << lane) - 1))] = i;
                ng += __popcll(ge);
                nart += __popcll(ar);
                neq += __popcll(eq);
            }
            if (lane == 0) { sh->ng = ng; sh->nart = nart; sh->neq = neq; }
        }
        __syncthreads();
        P.N = n + sh->ng;
        P.C = P.N + 1;
        P.ld = tableau_ld(P.C, int(sizeof(T)));
        P.nart = sh->nart;
        const int64_t tab_bytes = int64_t(m + 1) * P.ld * int64_t(sizeof(T));
        const bool in_lds = !a.force_hbm && L.tab + tab_bytes <= int64_t(a.lds_bytes);
        if (!in_lds && (!a.scratch || tab_bytes > a.slot_bytes)) {
            reject_lp<T, NT>(P, a);
        } else if (in_lds) {
            P.tab = reinterpret_cast<T *>(smem + L.tab);
            solve_lp<T, NT>(P, a, 3);
        } else {
            P.tab = reinterpret_cast<T *>(a.scratch + int64_t(blockIdx.x) * a.slot_bytes);
            solve_lp<T, NT>(P, a, 2);
        }
        item = sh->next;
        __syncthreads();
    }
    if (tid == 0) finish_launch(a.queue, a.done, a.reset_extra);
}

__global__ void zero_i32_kernel(int32_t *p, int count)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void set_i32_kernel(int32_t *p, int32_t value)
{
    if (threadIdx.x == 0) *p = value;
}

template <typename T, int NT>
hipError_t launch_t(const SolveArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((simplex_kernel<T, NT>), dim3(grid), dim3(NT), a.lds_bytes, s, a);
    return hipGetLastError();
}

template <typename T, int NT>
int occ_t(int lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void *)simplex_kernel<T, NT>,
                                                     NT, lds) != hipSuccess)
        return 0;
    return blocks;
}

}  // namespace

hipError_t launch_zero_i32(int32_t *p, int count, hipStream_t s)
{
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_set_i32(int32_t *p, int32_t value, hipStream_t s)
{
    hipLaunchKernelGGL(set_i32_kernel, dim3(1), dim3(64), 0, s, p, value);
    return hipGetLastError();
}

hipError_t launch_simplex(bool fp32, int nt, const SolveArgs &a, int grid, hipStream_t s)
{
    switch (nt) {
    case 64: return fp32 ? launch_t<float, 64>(a, grid, s) : launch_t<double, 64>(a, grid, s);
    case 128: return fp32 ? launch_t<float, 128>(a, grid, s) : launch_t<double, 128>(a, grid, s);
    case 256: return fp32 ? launch_t<float, 256>(a, grid, s) : launch_t<double, 256>(a, grid, s);
    case 512: return fp32 ? launch_t<float, 512>(a, grid, s) : launch_t<double, 512>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

int64_t simplex_ctrl_bytes(bool fp32) { return fp32 ? sizeof(Ctrl<float>) : sizeof(Ctrl<double>); }

hipError_t simplex_configure(int max_lds)
{
    const void *fns[] = {
        (const void *)simplex_kernel<float, 64>, (const void *)simplex_kernel<double, 64>,
        (const void *)simplex_kernel<float, 128>, (const void *)simplex_kernel<double, 128>,
        (const void *)simplex_kernel<float, 256>, (const void *)simplex_kernel<double, 256>,
        (const void *)simplex_kernel<float, 512>, (const void *)simplex_kernel<double, 512>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int simplex_blocks_per_cu(bool fp32, int nt, int lds)
{
    switch (nt) {
    case 64: return fp32 ? occ_t<float, 64>(lds) : occ_t<double, 64>(lds);
    case 128: return fp32 ? occ_t<float, 128>(lds) : occ_t<double, 128>(lds);
    case 256: return fp32 ? occ_t<float, 256>(lds) : occ_t<double, 256>(lds);
    case 512: return fp32 ? occ_t<float, 512>(lds) : occ_t<double, 512>(lds);
    default: return 0;
    }
}

}  // namespace lpb
