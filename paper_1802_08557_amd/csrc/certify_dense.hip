// certify_dense.hip -- the FP64 certificate of a final basis for batches of
// small LPs with their own constraint matrices (at most 64 rows and 64
// columns each, every A at most 64 * 40 entries): one wavefront per LP, the
// LP's whole input prefetched into registers one LP ahead and its A staged in
// LDS column-major, so every access of the certificate after the first load
// is an LDS or register access.
//
// The certificate is the one of certify_kernels.hip (and computes the same
// values in the same order): T = the rows whose slack/surplus is non-basic,
// S = the basic structurals; B_TS (sign-normalised) is LU-factorised with
// partial pivoting by wavefront max (lane t holds row t, column-major in LDS,
// rows not swapped); x_S = B_TS^-1 b_T and y_T = B_TS^-T c_S; the primal
// check covers x_S and every non-tight row's slack, the dual check every
// non-basic structural's reduced cost and the sign of every tight row's dual;
// an LP reported unbounded needs its ray B^-1 a_q to keep every basic
// variable and non-tight row feasible and to raise the objective.  A basis
// that passes writes its FP64 x and objective; any other goes to the FP64
// re-solve list.
//
// Streaming: the work item after the current one is known (blockIdx.x + G
// first, then from an atomic counter), and its A (flat row-major, element
// lane + 64 t in register t), b, c, sense and basis are loaded by unconditional
// buffer loads whose range check returns 0 past the LP's end, while the
// current LP is certified -- the HBM read of A, not the dependent chain of the
// certificate, bounds the kernel.
#include <math.h>

#include "device_common.h"
#include "internal.h"

namespace lpb {
namespace {

constexpr int kTightD = 32, kDeadD = 64;
constexpr int DPF = 40;  // doubles of A per lane: LPs of at most 64 * 40 entries

__device__ __forceinline__ void dsync() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }
__device__ __forceinline__ bool dall(bool v) { return __ballot(!v) == 0; }

// Column stride of the staged A: the smallest odd number of 16-byte units that
// holds m rows (lanes walking different columns of one row, or one column's
// rows, spread over the banks).
__host__ __device__ constexpr int dense_ldm(int m) { return 2 * (((m + 1) / 2) | 1); }

struct DFetch {
    int64_t k, ro, co;
    int m, n;
    double av[DPF];
    double bv, cv;
    int sv, bas, st, en;
};

__device__ __forceinline__ void dense_fetch(const CertArgs &a, int64_t item, DFetch &F)
{
    const int lane = threadIdx.x;
    const int64_t k = item;
    F.k = k;
    int m, n;
    int64_t aoff;
    if (a.um > 0) {
        m = a.um; n = a.un;
        aoff = k * int64_t(m) * n;
        F.ro = k * m;
        F.co = k * n;
    } else {
        const int mk = a.m[k], nk = a.n[k];
        const int64_t ak = a.aoff[k], rk = a.roff[k], ck = a.coff[k];
        m = uniform(mk); n = uniform(nk);
        aoff = uniform64(ak);
        F.ro = uniform64(rk);
        F.co = uniform64(ck);
    }
    F.m = m; F.n = n;
    const __amdgpu_buffer_rsrc_t ra = buffer_over(a.A + aoff, m * n * int(sizeof(double)));
#pragma unroll
    for (int t = 0; t < DPF; ++t) F.av[t] = buffer_f64(ra, (lane + 64 * t) * int(sizeof(double)));
    F.bv = buffer_f64(buffer_over(a.b + F.ro, m * int(sizeof(double))), lane * int(sizeof(double)));
    F.cv = buffer_f64(buffer_over(a.c + F.co, n * int(sizeof(double))), lane * int(sizeof(double)));
    F.sv = int(int8_t(__builtin_amdgcn_raw_buffer_load_b8(buffer_over(a.sense + F.ro, m), lane, 0, 0)));
    F.bas = int(__builtin_amdgcn_raw_buffer_load_b32(buffer_over(a.basis + F.ro, m * 4), lane * 4, 0, 0));
    F.st = int(__builtin_amdgcn_raw_buffer_load_b32(buffer_over(a.status + k, 4), 0, 0, 0));
    F.en = int(__builtin_amdgcn_raw_buffer_load_b32(buffer_over(a.enter + k, 4), 0, 0, 0));
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void certify_dense_kernel(CertArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x;
    constexpr int CG = 8;
    // LDS: this wavefront's A (column-major, a.wave_bytes bytes sized for the
    // launch's largest LP), then its certificate arrays.
    double *tab = reinterpret_cast<double *>(smem);
    char *my = smem + a.wave_bytes;
    const WaveCertLayout L = wave_cert_layout(64, 64, a.kl);
    int *rowfl = reinterpret_cast<int *>(my + L.rowf);
    int *colfl = reinterpret_cast<int *>(my + L.colf);
    int *tlist = reinterpret_cast<int *>(my + L.tlist);
    int *slist = reinterpret_cast<int *>(my + L.slist);
    int *order = reinterpret_cast<int *>(my + L.order);
    double *xsv = reinterpret_cast<double *>(my + L.xs);
    double *yv = reinterpret_cast<double *>(my + L.yv);
    double *M = reinterpret_cast<double *>(my + L.mat);
    const int64_t total = a.num;
    const int64_t G = gridDim.x;
    int64_t cur = blockIdx.x, nxt = blockIdx.x + G;
    DFetch F;
    if (cur < total) dense_fetch(a, cur, F);
    while (cur < total) {
        int qv = 0;
        if (lane == 0) qv = int(atomicInc(reinterpret_cast<unsigned *>(a.queue), 0xffffffffu));
        const int64_t k = F.k;
        const int m = uniform(F.m), n = uniform(F.n), ldm = dense_ldm(m);
        const int64_t co = F.co;
        // A scattered from flat row-major order into the columns (element
        // f = lane + 64 t: row f / n, column f % n); entries past m * n read 0.
        bool bad = false;
        {
            const int mn = m * n;
            const int dq = 64 / n, dr = 64 - dq * n;
            int ri = lane / n, cj = lane - ri * n;
#pragma unroll
            for (int t = 0; t < DPF; ++t) {
                if (lane + 64 * t < mn) tab[cj * ldm + ri] = F.av[t];
                ri += dq;
                cj += dr;
                if (cj >= n) { cj -= n; ++ri; }
            }
        }
        const double bi = fresh_copy(F.bv), cj = fresh_copy(F.cv);
        const int si = F.sv, v = F.bas, st0 = uniform(F.st), enter_q = uniform(F.en);
        // The registers of F are free: start loading the next LP (the last LP
        // of a wavefront reloads itself, so the loads are unconditional).
        dense_fetch(a, nxt < total ? nxt : cur, F);

        int cert = 0;
        bool fallback = !(st0 == kOptimal || st0 == kUnbounded);
        const bool work = st0 == kOptimal || st0 == kUnbounded;
        if (a.viol && lane == 0) a.viol[k] = kBig;  // until the primal check counts them
        double *x = a.x + co;
        if (work) {
            // Rows: sign normalisation and the tight set; columns: the basic set.
            int sen = si;
            const bool neg = bi < 0.0;
            if (neg && sen != kEQ) sen = (sen == kLE) ? kGE : kLE;
            if (lane < m) rowfl[lane] = (neg ? kRowNeg : 0) | (sen << 1) | kTightD;
            // x = 0 feasible (every normalised row <= or b = 0): a ray alone
            // then proves the LP unbounded.
            const bool origin = !__ballot(lane < m && sen != kLE && bi != 0.0);
            if (lane < n) colfl[lane] = 0;
            dsync();
            if (lane < m) {
                if (v < -1 || v >= n + 2 * m) {
                    bad = true;
                } else if (v < 0) {
                    atomicOr(&rowfl[lane], kDeadD);
                    atomicAnd(&rowfl[lane], ~kTightD);
                } else if (v < n) {
                    colfl[v] = kTightD;
                } else if (v < n + m) {
                    atomicAnd(&rowfl[v - n], ~kTightD);
                } else {
                    atomicOr(&rowfl[v - n - m], kDeadD);
                    atomicAnd(&rowfl[v - n - m], ~kTightD);
                }
            }
            dsync();
            const int rf = lane < m ? rowfl[lane] : 0;
            const bool isbasic = lane < n && colfl[lane] != 0;
            const uint64_t tmask = __ballot(lane < m && (rf & kTightD));
            const uint64_t smask = __ballot(isbasic);
            const int kt = __popcll(tmask), K = __popcll(smask);
            const int KL = K | 1;  // M's column stride: odd, so row reads of M miss no bank twice
            const int tpos = (tmask >> lane) & 1 ? __popcll(tmask & lanemask_lt(lane)) : -1;
            const int spos = isbasic ? __popcll(smask & lanemask_lt(lane)) : -1;
            if (tpos >= 0) tlist[tpos] = lane;
            if (spos >= 0) slist[spos] = lane;
            dsync();
            const double bnorm = wave_max_f(lane < m ? fabs(bi) : 0.0), cnorm = wave_max_f(lane < n ? fabs(cj) : 0.0);
            const double tol_p = a.tol_feas * (1.0 + bnorm);
            const double tol_d = a.tol_opt * fmax(1.0, cnorm);
            bool ok = kt == K && K <= a.kl && __ballot(bad) == 0;
            const bool kfit = K <= a.kl;
            const int tl = (lane < K && kfit) ? tlist[lane] : 0;
            const int sl = (lane < K && kfit) ? slist[lane] : 0;
            const int rft = __shfl(rf, tl);
            const double sgt = (lane < K && kfit && (rft & kRowNeg)) ? -1.0 : 1.0;
            double rz = 0.0, cs = 0.0;
            int pos = kBig;  // step at which this lane's row became the pivot row
            int ordr = 0;    // lane p: the row chosen at step p
            double rinv = 0.0;  // lane p: 1 / U_pp, recorded by the LU's step p
            const double btl = __shfl(bi, tl), csl = __shfl(cj, sl);
            if (ok) {
                double am = 0.0;
                double colv = 0.0;
                for (int s0 = 0; s0 < K; s0 += CG) {
                    int ci[CG];
#pragma unroll
                    for (int q = 0; q < CG; ++q) ci[q] = lane_get(sl, s0 + q < K ? s0 + q : 0);
                    double vv[CG] = {};
                    if (lane < K) {
#pragma unroll
                        for (int q = 0; q < CG; ++q) vv[q] = (s0 + q < K) ? sgt * tab[ci[q] * ldm + tl] : 0.0;
                    }
                    if (s0 == 0) colv = (lane < K) ? vv[0] : 0.0;
#pragma unroll
                    for (int q = 0; q < CG; ++q)
                        if (s0 + q < K && lane < K) {
                            M[(s0 + q) * KL + lane] = vv[q];
                            am = fmax(am, fabs(vv[q]));
                        }
                }
                rz = (lane < K) ? sgt * btl : 0.0;
                cs = (lane < K) ? csl : 0.0;
                const double amax = wave_max_f(am);
                dsync();
                for (int p = 0; p < K; ++p) {
                    const double vp = (lane < K && pos == kBig) ? fabs(colv) : -1.0;
                    // Every lane's reciprocal, computed while the maximum is
                    // reduced: the pivot's is taken below, off the serial chain.
                    const double cinv = 1.0 / colv;
                    const double vmax = wave_max_f(vp);
                    if (!(vmax > 1e-13 * fmax(1.0, amax))) { ok = false; break; }
                    const int pl = __builtin_ctzll(__ballot(vp == vmax));
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
                    dsync();
                }
                if (!ok) cert |= LP_CERT_SINGULAR_BIT;
            }
            double xr = 0.0;  // lane p: x of the p-th basic structural
            if (ok) {
                // x_S (L z = P b_T, then U x = z) and y_T (U^T w = c_S, then
                // L^T v = w, y_t = v[pos_t]) side by side; 1 / U_pp comes from the LU (lane p).
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
                            mv[q] = M[p * KL + lane];
                            mu[q] = M[lane * KL + op[q]];
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
                            mv[q] = M[p * KL + lane];
                            ml[q] = M[lane * KL + op[q]];
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
                dsync();

                // Primal certificate: x_S and every non-tight row's slack (lane i: row i).
                bool pf = !(lane < K) || xr >= -tol_p;
                int nviol = __popcll(__ballot(!pf));
                {
                    bool rowok = true;
                    const bool act = lane < m && !(rf & kTightD);
                    double ax[4] = {0.0, 0.0, 0.0, 0.0};
                    for (int s0 = 0; s0 < K; s0 += CG) {
                        int sidx[CG];
                        double xq[CG];
#pragma unroll
                        for (int q = 0; q < CG; ++q) {
                            sidx[q] = lane_get(sl, s0 + q < K ? s0 + q : 0);
                            xq[q] = lane_get(xr, s0 + q < K ? s0 + q : 0);
                        }
                        if (act) {
                            double av[CG];
#pragma unroll
                            for (int q = 0; q < CG; ++q) av[q] = tab[sidx[q] * ldm + lane];
#pragma unroll
                            for (int q = 0; q < CG; ++q)
                                if (s0 + q < K) ax[q & 3] = fma(av[q], xq[q], ax[q & 3]);
                        }
                    }
                    if (act) {
                        const double sg = (rf & kRowNeg) ? -1.0 : 1.0;
                        const double r = sg * (bi - ((ax[0] + ax[1]) + (ax[2] + ax[3])));
                        const int rs = (rf >> 1) & 3;
                        if ((rf & kDeadD) || rs == kEQ) rowok = fabs(r) <= tol_p;
                        else if (rs == kLE) rowok = r >= -tol_p;
                        else if (rs == kGE) rowok = -r >= -tol_p;
                    }
                    pf &= rowok;
                    nviol += __popcll(__ballot(!rowok));
                }
                const bool primal_ok = dall(pf);
                if (primal_ok) cert |= LP_CERT_PRIMAL_OK_BIT;
                if (a.viol && lane == 0) a.viol[k] = nviol;

                if (st0 == kOptimal && primal_ok) {
                    // Dual certificate: reduced costs of every non-basic column (lane j).
                    bool df = true;
                    const bool act = lane < n && spos < 0;
                    double ya[4] = {0.0, 0.0, 0.0, 0.0};
                    for (int t0 = 0; t0 < K; t0 += CG) {
                        int ti[CG];
                        double yq[CG];
#pragma unroll
                        for (int q = 0; q < CG; ++q) {
                            ti[q] = lane_get(tl, t0 + q < K ? t0 + q : 0);
                            yq[q] = lane_get(ysg, t0 + q < K ? t0 + q : 0);
                        }
                        if (act) {
                            double av[CG];
#pragma unroll
                            for (int q = 0; q < CG; ++q) av[q] = tab[lane * ldm + ti[q]];
#pragma unroll
                            for (int q = 0; q < CG; ++q)
                                if (t0 + q < K) ya[q & 3] = fma(yq[q], av[q], ya[q & 3]);
                        }
                    }
                    if (act) df &= cj - ((ya[0] + ya[1]) + (ya[2] + ya[3])) <= tol_d;
                    if (lane < K) {
                        const int rs = (rft >> 1) & 3;
                        if (rs == kLE) df &= -yt <= tol_d;
                        else if (rs == kGE) df &= yt <= tol_d;
                    }
                    if (dall(df)) cert |= LP_CERT_DUAL_OK_BIT;
                } else if (st0 == kUnbounded && (primal_ok || origin)) {
                    // Ray of the entering variable q: w = B^-1 a_q, d_S = -w.
                    const int q = enter_q;
                    const bool qbasic = q >= 0 && q < n && __shfl(spos, q) >= 0;
                    bool rf2 = q >= 0 && q < n + m && !qbasic;
                    int tr = -1;
                    double sq = 0.0;
                    if (rf2 && q >= n) {
                        tr = __shfl(tpos, q - n);
                        const int rs = (__shfl(rf, q - n) >> 1) & 3;
                        rf2 = tr >= 0 && rs != kEQ;
                        sq = (rs == kLE) ? 1.0 : -1.0;
                    }
                    if (rf2) {
                        double rw = 0.0;
                        if (lane < K) rw = (q < n) ? sgt * tab[q * ldm + tl] : (lane == tr ? sq : 0.0);
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
                        double gain = (lane < K) ? __shfl(cj, sl) * -wd : 0.0;
                        dsync();
                        if (lane < K) xsv[lane] = wd;  // x_S is no longer needed
                        dsync();
                        if (lane < m && !(rf & kTightD)) {
                            const double sg = (rf & kRowNeg) ? -1.0 : 1.0;
                            double ad = (q < n) ? tab[q * ldm + lane] : 0.0;
                            for (int s2 = 0; s2 < K; ++s2) ad = fma(tab[slist[s2] * ldm + lane], -xsv[s2], ad);
                            const double dr = -sg * ad;
                            const int rs = (rf >> 1) & 3;
                            if ((rf & kDeadD) || rs == kEQ) ok2 &= fabs(dr) <= tol_r;
                            else if (rs == kLE) ok2 &= dr >= -tol_r;
                            else if (rs == kGE) ok2 &= -dr >= -tol_r;
                        }
                        double g = gain;
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o);
                        const double cq = (q < n) ? __shfl(cj, q) : 0.0;
                        if (dall(ok2) && cq + g > tol_d) cert |= LP_CERT_RAY_OK_BIT;
                    }
                }
            }
            const bool passed = (st0 == kOptimal) ? (cert & LP_CERT_DUAL_OK_BIT) && (cert & LP_CERT_PRIMAL_OK_BIT)
                                                  : (cert & LP_CERT_RAY_OK_BIT) != 0;
            fallback = !passed;
            if (passed && st0 == kOptimal) {
                const double xj = (spos >= 0) ? xsv[spos] : 0.0;
                if (lane < n) x[lane] = xj;
                double z = (lane < n) ? fma(cj, xj, 0.0) : 0.0;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) z += __shfl_xor(z, o);
                if (lane == 0) a.obj[k] = z;
            } else if (passed) {
                if (lane < n) x[lane] = __builtin_nan("");
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
        dsync();
        cur = nxt;
        nxt = 2 * G + lane_get(qv, 0);
    }
    if (lane == 0) finish_launch(a.queue, a.done, nullptr);
}

}  // namespace

// Bytes of the staged A of an LP of at most m_max x n_max (CertArgs.wave_bytes
// of the dense kernel), and the LDS of its one-wavefront workgroup with LU
// blocks up to kl x kl.
int64_t certify_dense_a_bytes(int m_max, int n_max) { return align16(int64_t(n_max) * dense_ldm(m_max) * 8); }
int64_t certify_dense_lds_bytes(int m_max, int n_max, int kl)
{
    return certify_dense_a_bytes(m_max, n_max) + wave_cert_layout(64, 64, kl).end;
}

int certify_dense_prefetch_elems() { return 64 * DPF; }

hipError_t launch_certify_dense(const CertArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(certify_dense_kernel, dim3(grid), dim3(64), a.lds_bytes, s, a);
    return hipGetLastError();
}

int certify_dense_blocks_per_cu(int lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void *)certify_dense_kernel, 64, lds) !=
        hipSuccess)
        return 0;
    return blocks;
}

hipError_t certify_dense_configure(int max_lds)
{
    return hipFuncSetAttribute((const void *)certify_dense_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               max_lds);
}

}  // namespace lpb
