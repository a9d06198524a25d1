// wave_kernels.hip -- one 64-wide wavefront per LP for small tableaux.
//
// For LPs with at most 63 non-basic columns and 64*RB rows the whole solve runs
// in a single wavefront with no workgroup barrier:
//   * lane j owns column j: its non-basic variable nonb (Bland index), its
//     objective-row entry d_j (lane N holds minus the objective value) and, during
//     a pivot, its pivot-row entry prow_j;
//   * lane i (+64 r) owns row i: its basic variable, sign/sense flags and its
//     pivot-column entry pcol_i;
//   * the constraint rows live in LDS, column-major (lane j's column is
//     contiguous) with a column stride of an odd number of 16-byte units.
// Step 1 is a wavefront DPP/permlane reduction over the lanes' reduced costs;
// Step 2 reads the entering column and the rhs column (contiguous, one element
// per lane) and reduces the ratios; Step 3 sweeps each lane's column in 16-byte
// vectors, sixteen rows per group -- all reads, then the fma, then all writes --
// with each row's pivot-column entry read from its owning lane (readlane),
// then rewrites the swapped column and the pivot row.
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
    T *tab;  // column-major: element (i, j) at tab[j * ldm + i]
    int rowf[RB], basis[RB];
    T pcol[RB];
    int nonb;  // this lane's column
    T d;       // this lane's objective-row entry
    int iters, it1, degp, cap;
};

// Rows r0 .. r0+R-1 of one 16-byte vector of this lane's column:
// v[r] = fma(-pcol_row, prow, v[r]).  Rows at or past m are padding that is
// never read back, so whatever pivot-column entry they pick up is irrelevant.
template <typename T, int RB, typename V>
__device__ __forceinline__ void update_vec(V &v, int r0, const T (&pcol)[RB], T prow)
{
    constexpr int R = 16 / int(sizeof(T));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T f = row_get<RB>(pcol, r0 + r);
        v[r] = fma(-f, prow, v[r]);
    }
}

template <typename T, int RB>
__device__ __forceinline__ void pivot(WaveLP<T, RB> &P, int l, int e)
{
    using V = T __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int R = 16 / int(sizeof(T));
    constexpr int G = 16 / R;  // vectors per group of 16 rows
    const int lane = threadIdx.x;
    const int m = P.m, C = P.C, ldm = P.ldm;
    T *tab = P.tab;
    const T pe = row_get<RB>(P.pcol, l);
    T prow = T(0);
    if (lane < C) prow = (lane == e) ? T(1) / pe : tab[lane * ldm + l] / pe;
    const T de = lane_get(P.d, e);
    if (lane < C) P.d = fma(-de, prow, (lane == e) ? T(0) : P.d);
    // Sweep this lane's column in 16-byte vectors, G vectors (16 rows) per
    // group; the pivot row and the swapped column are rewritten afterwards.
    if (lane < C) {
        V *col = reinterpret_cast<V *>(tab + lane * ldm);
        const int nv = (m + R - 1) / R;
        int k0 = 0;
        for (; k0 + G <= nv; k0 += G) {
            V v[G];
#pragma unroll
            for (int g = 0; g < G; ++g) v[g] = col[k0 + g];
#pragma unroll
            for (int g = 0; g < G; ++g) update_vec<T, RB>(v[g], (k0 + g) * R, P.pcol, prow);
#pragma unroll
            for (int g = 0; g < G; ++g) col[k0 + g] = v[g];
        }
        for (; k0 < nv; ++k0) {
            V v = col[k0];
            update_vec<T, RB>(v, k0 * R, P.pcol, prow);
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
    const int bl = row_get<RB>(P.basis, l);
    const int ne = lane_get(P.nonb, e);
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (lane + 64 * r == l) P.basis[r] = ne;
    if (lane == e) P.nonb = bl;
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

template <typename T, int RB>
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
        const int e = price<T>(lane < N && P.d > eps_opt && P.nonb < nm, P.d, P.nonb, bland);
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
            if (i < m) { a = tab[e * ldm + i]; bi = tab[N * ldm + i]; }
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
        pivot<T, RB>(P, l, e);
        ++P.iters;
    }
}

// Bytes of LDS the wave kernel keeps in front of the tableau.
__host__ __device__ constexpr int64_t wave_aux_bytes(int rb, int64_t tsize)
{
    return align16(4 * 64 * rb) + align16(tsize * 64);
}

template <typename T, int RB>
__global__ __launch_bounds__(64) void simplex_wave_kernel(SolveArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x;
    int *colrow = reinterpret_cast<int *>(smem);
    T *xv = reinterpret_cast<T *>(smem + align16(4 * 64 * RB));
    const int64_t aux = wave_aux_bytes(RB, sizeof(T));
    int64_t item = blockIdx.x;
    while (item < a.num) {
        int nxt = 0;
        if (lane == 0) nxt = int(gridDim.x) + atomicAdd(a.queue, 1);
        const int64_t k = a.ids ? int64_t(a.ids[item]) : item;
        WaveLP<T, RB> P;
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
        const int m = P.m, n = P.n;

        // A1: sign-normalise and classify rows; surplus columns by ballot.
        bool bad = false;
        double bv[RB];
        int sc[RB];
        int ng = 0, nart = 0, neq = 0;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = lane + 64 * r;
            int f = kRowPad;
            double bi = 0.0;
            if (i < m) {
                bi = P.b[i];
                const int s = a.sense[P.ro + i];
                bad |= !isfinite(bi) || s < kLE || s > kEQ;
                const bool neg = bi < 0.0;
                int sen = (s < kLE || s > kEQ) ? kLE : s;
                if (neg && sen != kEQ) sen = (sen == kLE) ? kGE : kLE;
                f = (neg ? kRowNeg : 0) | (sen << 1);
            }
            bv[r] = bi;
            P.rowf[r] = f;
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
        P.C = P.N + 1;
        P.ldm = col_stride<T>(m);
        P.nart = nart;
        const int64_t need = aux + int64_t(P.C) * P.ldm * int64_t(sizeof(T));
        if (P.C > 64 || m > 64 * RB || need > a.lds_bytes) {
            if (lane == 0) {
                const int slot = atomicAdd(a.defer_count, 1);
                a.defer_ids[slot] = int32_t(k);
            }
            item = lane_get(nxt, 0);
            continue;
        }
        const int N = P.N, C = P.C, ldm = P.ldm;
        T *tab = reinterpret_cast<T *>(smem + aux);
        P.tab = tab;

        // A2: index arrays and the tableau rows (U rows of A in flight).
        P.nonb = kBig;
        double cj = 0.0;
        if (lane < n) {
            P.nonb = lane;
            cj = P.c[lane];
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
            // A (m x n, contiguous) copied with UB independent loads per lane in
            // flight; row = (f + 0.5) / n in float is exact for f < 2^13.
            constexpr int UB = 16;
            const int mn = m * n;
            const float inv_n = 1.0f / float(n);
            for (int f0 = 0; f0 < mn; f0 += 64 * UB) {
                double av[UB];
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int f = f0 + 64 * u + lane;
                    av[u] = (f < mn) ? P.A[f] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int f = f0 + 64 * u + lane;
                    if (f < mn) {
                        const int i = int((float(f) + 0.5f) * inv_n);
                        const int j = f - i * n;
                        bad |= !isfinite(av[u]);
                        tab[j * ldm + i] = T(av[u]);
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
            // Surplus columns and the right-hand side, one row per lane.
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = lane + 64 * r;
                if (i < m) {
                    const double sg = (P.rowf[r] & kRowNeg) ? -1.0 : 1.0;
                    for (int g = 0; g < ng; ++g) tab[(n + g) * ldm + i] = (sc[r] == n + g) ? T(-1) : T(0);
                    tab[N * ldm + i] = T(sg * bv[r]);
                }
            }
        }
        const bool invalid = __ballot(bad) != 0;
        const double cnorm = wave_max(fabs(cj));
        double bm = 0.0;
#pragma unroll
        for (int r = 0; r < RB; ++r) bm = fmax(bm, fabs(bv[r]));
        const double bnorm = wave_max(bm);
        P.iters = 0; P.it1 = 0; P.degp = 0;
        P.cap = a.prm.max_iters > 0 ? a.prm.max_iters : 50 * (m + n + (m - neq) + nart);
        P.d = T(0);
        int status = kOptimal, enter = -1;

        if (invalid) {
            status = kInvalid;
        } else {
            if (nart > 0) {
                // Phase I objective row: sum of the artificial rows in row order.
                T acc = T(0);
                for (int i = 0; i < m; ++i) {
                    const int sen = (row_get<RB>(P.rowf, i) >> 1) & 3;
                    if (sen != kLE && lane < C) acc += tab[lane * ldm + i];
                }
                P.d = acc;
                const double dmax = wave_max(lane < N ? fabs(double(acc)) : 0.0);
                const double dscale = fmax(1.0, dmax);
                const int r = simplex<T, RB>(P, T(a.prm.tol_opt * dscale), a.prm, &enter);
                P.it1 = P.iters;
                enter = -1;
                if (r == kIterLimit) status = kIterLimit;
                else if (r == kUnbounded) status = kNumerical;
                else {
                    const double wstar = -double(lane_get(P.d, N));
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
            if (status == kOptimal) {
                // Phase II objective row: c priced out over the basis, rows in order.
                T cb[RB];
                uint64_t nz[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int bvr = P.basis[r];
                    cb[r] = (!(P.rowf[r] & (kRowDead | kRowPad)) && bvr < n) ? T(P.c[bvr]) : T(0);
                    nz[r] = __ballot(cb[r] != T(0));
                }
                T acc = (lane < N && P.nonb < n) ? T(P.c[P.nonb]) : T(0);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    uint64_t mk = nz[r];
                    while (mk) {
                        const int bit = __builtin_ctzll(mk);
                        mk &= mk - 1;
                        const T f = lane_get(cb[r], bit);
                        if (lane < C) acc = fma(-f, tab[lane * ldm + 64 * r + bit], acc);
                    }
                }
                P.d = acc;
                status = simplex<T, RB>(P, T(a.prm.tol_opt * fmax(1.0, cnorm)), a.prm, &enter);
            }
        }

        // A8: extraction through an LDS staging vector.
        if (lane < n) xv[lane] = T(0);
        if (status == kOptimal) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = lane + 64 * r;
                const int bvr = P.basis[r];
                if (i < m && bvr < n && !(P.rowf[r] & kRowDead)) xv[bvr] = tab[N * ldm + i];
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
                st[0] = P.it1;
                st[1] = P.iters - P.it1;
                st[2] = P.degp;
                st[3] = 0;
                st[4] = 0;
                st[5] = 0;
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
        item = lane_get(nxt, 0);
    }
}

template <typename T, int RB>
hipError_t launch_t(const SolveArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((simplex_wave_kernel<T, RB>), dim3(grid), dim3(64), a.lds_bytes, s, a);
    return hipGetLastError();
}

template <typename T, int RB>
int occ_t(int lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &blocks, (const void *)simplex_wave_kernel<T, RB>, 64, lds) != hipSuccess)
        return 0;
    return blocks;
}

}  // namespace

int64_t wave_lds_aux_bytes(int rb, bool fp32) { return wave_aux_bytes(rb, fp32 ? 4 : 8); }

hipError_t launch_simplex_wave(bool fp32, int rb, const SolveArgs &a, int grid, hipStream_t s)
{
    if (rb == 1) return fp32 ? launch_t<float, 1>(a, grid, s) : launch_t<double, 1>(a, grid, s);
    if (rb == 2) return fp32 ? launch_t<float, 2>(a, grid, s) : launch_t<double, 2>(a, grid, s);
    return hipErrorInvalidValue;
}

int simplex_wave_blocks_per_cu(bool fp32, int rb, int lds)
{
    if (rb == 1) return fp32 ? occ_t<float, 1>(lds) : occ_t<double, 1>(lds);
    if (rb == 2) return fp32 ? occ_t<float, 2>(lds) : occ_t<double, 2>(lds);
    return 0;
}

hipError_t simplex_wave_configure(int max_lds)
{
    const void *fns[] = {(const void *)simplex_wave_kernel<float, 1>,
                         (const void *)simplex_wave_kernel<double, 1>,
                         (const void *)simplex_wave_kernel<float, 2>,
                         (const void *)simplex_wave_kernel<double, 2>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lpb
