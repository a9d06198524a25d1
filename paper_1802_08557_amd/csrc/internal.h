// internal.h -- structures shared by the host runtime and the HIP kernels.
// Not part of the public ABI (include/lpbatch.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpb {

__host__ __device__ inline int64_t align16(int64_t v) { return (v + 15) & ~int64_t(15); }

// Tolerances and limits of one solve (the public lp_options with defaults filled in).
struct SolveParams {
    double tol_piv;    // a pivot-column entry must exceed this to be eligible (Step 2)
    double tol_opt;    // reduced costs above tol_opt * max(1, |c|_inf) may enter (Step 1)
    double tol_feas;   // Phase I optimum below -tol_feas * (1 + |b|_inf) means infeasible
    int32_t k_deg;     // consecutive degenerate pivots before Bland's rule; <= 0: never
    int32_t max_iters; // pivot cap over both phases; <= 0: 50 * (m + #columns)
    int32_t pricing;   // 0: Dantzig; 1: steepest edge (d_j^2 / (1 + |column j|^2))
};

// Everything one launch of the simplex kernel needs.  Device pointers unless noted.
struct SolveArgs {
    int64_t num;              // work items in this launch (upper bound if num_dev is set)
    const int32_t *ids;       // work item -> LP index; null: identity
    const int32_t *num_dev;   // optional device-side count: items = id_base + *num_dev
    int32_t id_base;
    const double *A, *b, *c;  // batch data, layout of include/lpbatch.h
    const int8_t *sense;
    int32_t um, un;           // > 0: every LP is um x un (offsets computed, m/n/offsets unused)
    int32_t shared;           // 1: A, b, sense hold one LP of m_full x un shared by all LPs
                              //   (c, x, status, obj and basis_out stay per LP)
    const int32_t *row_subset;// shared only, optional [num][um]: LP k's row r is row
    int32_t m_full;           //   row_subset[k*um + r] of the shared LP (um <= m_full);
                              //   an index outside [0, m_full) makes the LP INVALID_INPUT
    const int32_t *m, *n;     // per-LP sizes when not uniform
    const int64_t *aoff, *roff, *coff;
    int32_t *status;          // outputs
    double *x, *obj;
    int32_t *stats;           // optional [num_lps][8]
    int32_t *basis_out;       // optional [sum m]: final basis (Bland index, -1 dropped row)
    int32_t *enter_out;       // optional [num_lps]: entering Bland index at UNBOUNDED
    char *scratch;            // HBM tableau slots, one per workgroup of the launch
    int64_t slot_bytes;
    int32_t *queue;           // work counter (0 at launch)
    int32_t *done;            // finished workgroups (0 at launch); the last one to finish
                              // resets queue, done and reset_extra to 0 for the next launch
    int32_t *reset_extra;     // optional
    int32_t *defer_ids;       // wavefront kernel: LPs it could not take are appended here,
    int32_t *defer_count;     //   from defer_ids[defer_base] on (the workgroup kernel
    int32_t defer_base;       //   then drains them)
    int32_t lds_bytes;        // dynamic LDS of each workgroup
    int32_t force_hbm;        // 1: never keep the tableau in LDS
    int32_t refine_stats;     // 1: a re-solve -- pivots go to stats[4], stats[3] = 1
    // Warm start of a re-solve (wavefront kernel, FP64, all-<= LPs): LP k
    // starts from the final basis of a relaxation solved on warm_m of its rows
    // -- warm_basis[k*warm_m + r] is the Bland index (relaxation numbering) of
    // the variable basic in relaxation row r, which is row warm_rows[k*warm_m + r]
    // of the LP.  Structurals are pivoted in, then the dual simplex method
    // repairs primal feasibility; an LP the repair does not finish optimal is
    // deferred to the workgroup kernel, which solves it from the slack basis.
    const int32_t *warm_basis;
    const int32_t *warm_rows;
    int32_t warm_m;
    const int32_t *warm_viol; // optional [num]: rows the relaxation's optimum violates; more
    int32_t warm_max_viol;    //   than warm_max_viol sends the LP to the slack-basis solve
    SolveParams prm;
};

// One launch of the FP64 certificate kernel (certify_kernels.hip).
struct CertArgs {
    int64_t num;
    const double *A, *b, *c;
    const int8_t *sense;
    int32_t um, un;
    int32_t shared;           // as in SolveArgs (um = rows of the shared LP)
    const int32_t *row_subset;// optional: the basis came from a solve on these rows only,
    int32_t subset_m;         //   subset_m per LP (basis and enter use that LP's numbering)
    const int32_t *m, *n;
    const int64_t *aoff, *roff, *coff;
    int32_t *status;
    double *x, *obj;
    int32_t *stats;
    const int32_t *basis;     // final basis of the single-precision solve
    const int32_t *enter;     // entering variable at UNBOUNDED
    int32_t *fb_ids;          // LPs to re-solve in FP64 are appended here
    int32_t *fb_count;
    int32_t *viol;            // optional [num]: rows the basis's x violates (wavefront kernel)
    char *scratch;            // LU matrices too large for LDS, one slot per workgroup
    int64_t slot_bytes;
    int32_t *queue, *done;
    // Workgroup kernel, optional: work item t is LP order1[t] for t < n1, else
    // order2[t - n1] (largest LPs first, so the launch does not end on one);
    // NULL: item t is LP t.
    const int32_t *order1, *order2;
    int64_t n1;
    int32_t lds_bytes;
    double tol_feas, tol_opt; // certificate tolerances (relative, as in SolveParams)
    // Wavefront kernels only: LDS bytes per wavefront (the dense kernel: the
    // bytes of its staged A), LU blocks up to kl x kl kept in LDS (a larger
    // basis goes to the FP64 re-solve), and whether the shared constraint
    // matrix is copied into LDS.
    int32_t wave_bytes, kl, stage_a;
};

// LDS carve-up of one LP in the wavefront certificate kernel (byte offsets).
struct WaveCertLayout {
    int64_t rowf, tpos, colf, spos, tlist, slist, order, xs, yv, mat, end;
};

__host__ __device__ inline WaveCertLayout wave_cert_layout(int m, int n, int kl)
{
    WaveCertLayout L;
    int64_t o = 0;
    L.rowf = o; o = align16(o + 4 * int64_t(m));
    L.tpos = o; o = align16(o + 4 * int64_t(m));
    L.colf = o; o = align16(o + 4 * int64_t(n));
    L.spos = o; o = align16(o + 4 * int64_t(n));
    L.tlist = o; o += 256;
    L.slist = o; o += 256;
    L.order = o; o += 256;
    L.xs = o; o = align16(o + 8 * int64_t(kl));  // x_S and y_T: k <= kl entries
    L.yv = o; o = align16(o + 8 * int64_t(kl));
    L.mat = o; o = align16(o + 8 * int64_t(kl) * (kl | 1));  // column stride k | 1
    L.end = o;
    return L;
}

hipError_t launch_certify_wave(int waves, const CertArgs &a, int grid, hipStream_t s);
int certify_wave_blocks_per_cu(int waves, int lds_bytes);

// Dense certificate (certify_dense.hip): one wavefront per LP of at most 64 x
// 64 and certify_dense_prefetch_elems() entries, own A (not shared, not
// screened); wave_bytes = certify_dense_a_bytes(m_max, n_max), kl <= 64.
hipError_t launch_certify_dense(const CertArgs &a, int grid, hipStream_t s);
int certify_dense_blocks_per_cu(int lds_bytes);
int64_t certify_dense_a_bytes(int m_max, int n_max);
int64_t certify_dense_lds_bytes(int m_max, int n_max, int kl);
int certify_dense_prefetch_elems();
hipError_t certify_dense_configure(int max_lds);

hipError_t launch_certify(int nt, const CertArgs &a, int grid, hipStream_t s);
int certify_blocks_per_cu(int nt, int lds_bytes);
int64_t certify_lds_bytes(int m, int n, bool with_matrix);
hipError_t certify_configure(int max_lds);

// Warm-start network (mlp_kernels.hip).  One strided BF16 GEMM with a fused
// epilogue: C[i][j] = sum_k a[i*sai + k*sak] * b[k*sbk + j*sbj] (+ bias[j]);
// zeroed where mask[i*ldc + j] <= 0 when mask is set; stored as FP32 (c32)
// and/or rounded to BF16 (c16, after a ReLU when relu is set).
struct MlpGemm {
    int M, N, K;
    const uint16_t *a, *b;
    int64_t sai, sak, sbk, sbj;
    const float *bias, *mask;
    float *c32;
    uint16_t *c16;
    int64_t ldc;
    int relu;
};

struct MlpAdam {
    float lr, wd, beta1, beta2, eps, bc1, bc2;  // bc = 1 - beta^t
};

hipError_t launch_mlp_gemm(const MlpGemm &g, hipStream_t s);
hipError_t launch_to_bf16(const float *x, uint16_t *y, int64_t count, hipStream_t s);
hipError_t launch_bce(const float *S, const uint8_t *Y, int64_t B, int O, float *dS, uint16_t *dS16,
                      float *row_loss, float *loss, hipStream_t s);
hipError_t launch_colsum(const float *dZ, int64_t B, int N, float *db, hipStream_t s);
hipError_t launch_adamw(float *w, const float *g, float *m, float *v, uint16_t *w16, int64_t count,
                        const MlpAdam &h, const int64_t (&decay)[6], hipStream_t s);
hipError_t launch_cast_params(const float *w, uint16_t *w16, int64_t count, hipStream_t s);
hipError_t launch_topk(const float *S, int64_t B, int O, int k, int32_t *out, hipStream_t s);
// Fused inference (all layers and the top-k, tiles of 64 directions):
// scores [B][120] and/or topk [B][k] (either may be NULL).
hipError_t launch_mlp_infer(const float *dirs, int64_t B, const uint16_t *w16, const float *w32, float *scores,
                            int32_t *topk, int k, hipStream_t s);
hipError_t mlp_configure();

// Closed-form box LPs (hyperbox_kernels.hip).
hipError_t launch_hyperbox(int64_t num, int n, const double *lo, const double *hi, const double *l,
                           int shared_box, double *value, double *x, hipStream_t s);

// Power-of-two scaling (scale_kernels.hip).  um/un: uniform shape, or 0 with
// the per-LP shape and offset arrays; c_out may be NULL (c left alone).
// host_m / host_n: the shapes in host memory (read to size the launch).
hipError_t launch_scale(int64_t num, int32_t um, int32_t un, const int32_t *m, const int32_t *n,
                        const int64_t *aoff, const int64_t *roff, const int64_t *coff, const int32_t *host_m,
                        const int32_t *host_n, int32_t passes, const double *A, const double *b, const double *c,
                        double *A_out, double *b_out, double *c_out, int32_t *rexp, int32_t *cexp, hipStream_t s);
// out[i] = in[i] * 2^e[i] (period 0) or 2^e[i % period]; in may equal out.
hipError_t launch_ldexp(int64_t count, const double *in, const int32_t *e, int64_t period, double *out,
                        hipStream_t s);

// Bland index convention shared by every kernel: structural j -> j, the
// slack/surplus of row i -> n + i, the artificial of row i -> n + m + i.

// Statically allocated device scratch of lp_batch_solve_noalloc (noalloc.hip):
// 256 bytes of work counters, the deferred-LP list (kNoAllocMaxLps entries),
// then the workgroup kernel's tableau slots.
constexpr int64_t kNoAllocBytes = int64_t(16) << 20;
constexpr int64_t kNoAllocMaxLps = int64_t(1) << 20;
constexpr int64_t kNoAllocIdsAt = 256;
constexpr int64_t kNoAllocSlotsAt = kNoAllocIdsAt + 4 * kNoAllocMaxLps;
// Device address of this device's copy (the current device's).
hipError_t noalloc_scratch_address(void **ptr);

// Launchers (simplex_kernels.hip).  Return the hipError_t of the launch.
hipError_t launch_zero_i32(int32_t *p, int count, hipStream_t s);
hipError_t launch_set_i32(int32_t *p, int32_t value, hipStream_t s);
hipError_t launch_simplex(bool fp32, int nt, const SolveArgs &a, int grid, hipStream_t s);
// Workgroups of the simplex kernel that fit one CU with this LDS (occupancy query).
int simplex_blocks_per_cu(bool fp32, int nt, int lds_bytes);
// Bytes of the kernel's LDS control block for the given tableau precision.
int64_t simplex_ctrl_bytes(bool fp32);
// Allows every simplex kernel instantiation up to max_lds bytes of dynamic LDS.
hipError_t simplex_configure(int max_lds);

// One-wavefront-per-LP kernel (wave_kernels.hip) for LPs of at most 64
// non-basic columns and 64*rb rows (rb = 1 or 2).
// pf: the instantiation that prefetches each next LP's A into registers
// (LPs of at most wave_prefetch_elems() entries, A not row-gathered).
hipError_t launch_simplex_wave(bool fp32, int rb, bool pf, const SolveArgs &a, int grid, hipStream_t s);
// The warm-start (repair) instantiation: FP64, no prefetch; a.warm_basis set.
hipError_t launch_simplex_wave_warm(int rb, const SolveArgs &a, int grid, hipStream_t s);
int simplex_wave_warm_blocks_per_cu(int rb, int lds_bytes);
int simplex_wave_blocks_per_cu(bool fp32, int rb, bool pf, int lds_bytes);
int wave_prefetch_elems();
int64_t wave_lds_aux_bytes(int rb, bool gather);
// LDS bytes of a column-major wavefront tableau with m rows and `cols` columns.
int64_t wave_tab_bytes(int m, int cols, bool fp32);
hipError_t simplex_wave_configure(int max_lds);

// Size of the LDS control block + index arrays + pivot row/column buffers for an
// LP with m rows and at most ncol_max non-basic columns, and the byte offset where
// an LDS-resident tableau would start.  Host and device compute the same layout.

struct LdsLayout {
    int64_t ctrl, basis, nonb, rowf, colrow, pcol, prow, pcol2, prow2, pcol3, prow3, tab, end_aux;
};

// ctrl_bytes: size of the control block (type dependent, passed by the caller).
__host__ __device__ inline LdsLayout lds_layout(int m, int ncol_max, int64_t tsize, int64_t ctrl_bytes)
{
    LdsLayout L;
    L.ctrl = 0;
    L.basis = align16(ctrl_bytes);
    L.nonb = align16(L.basis + 4 * (int64_t)m);
    L.rowf = align16(L.nonb + 4 * (int64_t)ncol_max);
    L.colrow = align16(L.rowf + 4 * (int64_t)m);
    L.pcol = align16(L.colrow + 4 * (int64_t)m);
    L.prow = align16(L.pcol + tsize * (int64_t)(m + 1));
    L.pcol2 = align16(L.prow + tsize * (int64_t)(ncol_max + 1));
    L.prow2 = align16(L.pcol2 + tsize * (int64_t)(m + 1));
    L.pcol3 = align16(L.prow2 + tsize * (int64_t)(ncol_max + 1));
    L.prow3 = align16(L.pcol3 + tsize * (int64_t)(m + 1));
    L.tab = align16(L.prow3 + tsize * (int64_t)(ncol_max + 1));
    L.end_aux = L.tab;
    return L;
}

// Row stride (elements) of a workgroup-kernel tableau with C = (non-basic
// columns + 1) entries per row and tsize-byte entries: an odd number of
// 16-byte units, so every row starts 16-byte aligned (the pivot sweep moves
// 16 bytes per lane per access) and walking a column of an LDS-resident
// tableau spreads over the banks.
__host__ __device__ inline int tableau_ld(int C, int tsize)
{
    const int R = 16 / tsize;
    return R * (((C + R - 1) / R) | 1);
}

}  // namespace lpb
