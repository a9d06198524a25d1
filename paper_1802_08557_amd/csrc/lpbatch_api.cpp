// lpbatch_api.cpp -- host runtime behind include/lpbatch.h.
//
// Validates a batch, plans the launch (Alg. 1 of the paper sizes batches by
// device memory; here the device holds the whole batch, and the planner sizes
// the per-workgroup LDS budget, workgroup size and the number of resident
// workgroups), allocates grow-only scratch in the context and queues the
// kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lpbatch.h"
#include "internal.h"
#include "ctx.h"

namespace lpb {
thread_local std::string g_last_error;
}

namespace {

using lpb::fail;
using lpb::DevBuf;
using lpb::DeviceGuard;
using lpb::Timer;

lpb::SolveParams fill_params(const lp_options &o, bool fp32)
{
    lpb::SolveParams p;
    p.tol_piv = o.tol_piv > 0 ? o.tol_piv : (fp32 ? 1e-6 : 1e-9);
    p.tol_opt = o.tol_opt > 0 ? o.tol_opt : (fp32 ? 1e-6 : 1e-9);
    p.tol_feas = o.tol_feas > 0 ? o.tol_feas : (fp32 ? 1e-6 : 1e-9);
    p.k_deg = o.k_deg == 0 ? 50 : o.k_deg;
    p.max_iters = o.max_iters;
    p.pricing = o.pricing;
    return p;
}

// A validated batch as the planner sees it.
struct Plan {
    int64_t num;
    bool uniform;
    int32_t m0, n0, m_max, n_max;
    int64_t mn_max;
    bool fp32;
    int64_t ts;
};

// Counters of one solve pass (wavefront kernel + workgroup kernel).
struct PassCounters {
    int32_t *wq, *wd;  // wavefront queue / finished
    int32_t *bq, *bd;  // workgroup queue / finished
    int32_t *defer;    // LPs deferred by the wavefront kernel
};

bool wave_fit(const lp_ctx *ctx, int64_t mk, int64_t nk, bool fp32, bool gather)
{
    return nk <= 64 && mk <= 128 &&
           lpb::wave_lds_aux_bytes(mk > 64 ? 2 : 1, gather) + lpb::wave_tab_bytes(int(mk), int(nk), fp32) <=
               ctx->max_lds;
}

// Queues one solve pass.  The LPs are either the n_wave + n_block LPs given by
// host-built id lists already on the device (wave_ids, and block ids at the
// front of defer_ids), or -- when list_count is set -- the device list
// list_ids[0 .. *list_count), all offered to the wavefront kernel first.
// LDS a workgroup-kernel tableau may take.  By default at most a third of
// the CU's LDS, so that three or more workgroups share a CU and hide each
// other's latency; a larger tableau streams from its device-memory slot
// instead.  LP_PLACE_LDS asks for LDS whenever the tableau fits at all.
int64_t lds_budget(const lp_ctx *ctx, int placement)
{
    return placement == LP_PLACE_LDS ? ctx->max_lds : ctx->max_lds / 3;
}

// LDS for one workgroup of the workgroup kernel that keeps per_cu of them
// resident: when registers already cap a CU at per_cu workgroups, each may
// take the CU's LDS / per_cu, and every LP whose tableau fits there next to
// the index arrays is then solved from LDS instead of a device-memory slot.
int64_t lds_share(const lp_ctx *ctx, bool fp32, int nt, int64_t lds, int per_cu)
{
    const int64_t share = std::min<int64_t>(ctx->max_lds, (int64_t(ctx->lds_per_cu) / per_cu) & ~int64_t(255));
    if (share <= lds) return lds;
    return lpb::simplex_blocks_per_cu(fp32, nt, int(share)) == per_cu ? share : lds;
}

// One persistent launch of the wavefront kernel over ids[0 .. num) (or the
// device list ids[0 .. *list_count)); LPs it cannot take are appended to
// defer_ids from defer_base on.
int launch_wave(lp_ctx *ctx, bool fp32, const lpb::SolveArgs &a, PassCounters pc, const int32_t *ids, int64_t num,
                const int32_t *list_count, int wm_max, int wn_max, int32_t *defer_ids, int32_t defer_base,
                hipStream_t stream, bool timing, const char *name)
{
    const int rb = wm_max > 64 ? 2 : 1;
    lpb::SolveArgs w = a;
    w.num = num;
    w.ids = ids;
    w.num_dev = list_count;
    w.id_base = 0;
    w.queue = pc.wq;
    w.done = pc.wd;
    w.reset_extra = const_cast<int32_t *>(list_count);  // nothing reads it after this launch
    w.defer_ids = defer_ids;
    w.defer_count = pc.defer;
    w.defer_base = defer_base;
    // Budget for the common case of no surplus columns; an LP needing more is deferred.
    const bool gather = a.shared && a.row_subset;
    const int64_t lds = lpb::wave_lds_aux_bytes(rb, gather) + lpb::wave_tab_bytes(wm_max, wn_max, fp32);
    w.lds_bytes = int32_t(lds);
    // Prefetching A one LP ahead (measured faster for 50 x 50 in both
    // precisions) when every LP's A fits the prefetch registers; larger or
    // row-gathered LPs take the leaner instantiation, which runs more
    // wavefronts per SIMD.
    const bool warm = a.warm_basis != nullptr && !fp32;
    const bool pf = int64_t(wm_max) * wn_max <= lpb::wave_prefetch_elems() && !gather && !warm;
    const int per_cu = warm ? lpb::simplex_wave_warm_blocks_per_cu(rb, int(lds))
                            : lpb::simplex_wave_blocks_per_cu(fp32, rb, pf, int(lds));
    if (per_cu < 1) return fail(LP_ERR_HIP, "occupancy query failed for the wavefront kernel");
    const int64_t grid = std::min<int64_t>(num, int64_t(per_cu) * ctx->num_cu);
    Timer t(ctx, timing, stream, name);
    if (warm) HIP_TRY(lpb::launch_simplex_wave_warm(rb, w, int(grid), stream));
    else HIP_TRY(lpb::launch_simplex_wave(fp32, rb, pf, w, int(grid), stream));
    t.done();
    return LP_OK;
}

// slot_mem / slot_cap: device memory for the workgroup kernel's tableau slots
// given by the caller (the grid shrinks to what fits); NULL: the context's
// scratch, grown as needed.
int queue_pass(lp_ctx *ctx, const Plan &P, lpb::SolveArgs a, const lp_options &opts, PassCounters pc,
               const int32_t *wave_ids, int64_t n_wave, int wm_max, int wn_max, int64_t n_block,
               int32_t *defer_ids, const int32_t *list_ids, const int32_t *list_count,
               hipStream_t stream, bool timing, const char *wname, const char *bname,
               char *slot_mem = nullptr, int64_t slot_cap = 0)
{
    const bool fp32 = P.fp32;
    const int64_t ts = P.ts;
    if (n_wave > 0) {
        int rc = launch_wave(ctx, fp32, a, pc, list_count ? list_ids : wave_ids, list_count ? P.num : n_wave,
                             list_count, wm_max, wn_max, defer_ids, int32_t(n_block), stream, timing, wname);
        if (rc != LP_OK) return rc;
    }
    // Workgroup kernel: the LPs given to it plus the ones the wavefront deferred.
    const int ncol_worst = P.n_max + P.m_max;
    lpb::LdsLayout L = lpb::lds_layout(P.m_max, ncol_worst, ts, lpb::simplex_ctrl_bytes(fp32));
    // Tableau budget for the common case of no surplus columns (every row <= after
    // normalisation); LPs with more columns than budgeted move to HBM by themselves.
    const int64_t tab_common = int64_t(P.m_max + 1) * lpb::tableau_ld(P.n_max + 1, int(ts)) * ts;
    const int64_t tab_worst = int64_t(P.m_max + 1) * lpb::tableau_ld(ncol_worst + 1, int(ts)) * ts;
    const int64_t cells = int64_t(P.m_max + 1) * (P.n_max + 1);
    int nt = opts.block_threads;
    if (!nt) nt = cells <= 64 * 64 ? 64 : (cells <= 256 * 256 ? 256 : 512);
    int64_t lds = L.tab;
    const bool want_lds = opts.placement != LP_PLACE_HBM && L.tab + tab_common <= lds_budget(ctx, opts.placement);
    if (want_lds) lds = L.tab + tab_common;
    if (lds > ctx->max_lds)
        return fail(LP_ERR_ARG, "LP of %d rows x %d columns needs %lld bytes of LDS for its index "
                    "arrays (device limit %d)", P.m_max, ncol_worst, (long long)lds, ctx->max_lds);
    a.force_hbm = opts.placement == LP_PLACE_HBM;
    const int per_cu = lpb::simplex_blocks_per_cu(fp32, nt, int(lds));
    if (per_cu < 1) return fail(LP_ERR_HIP, "occupancy query failed for %d threads, %lld B LDS", nt, (long long)lds);
    if (!a.force_hbm) lds = lds_share(ctx, fp32, nt, lds, per_cu);
    a.lds_bytes = int32_t(lds);
    // When the wavefront kernel was offered every LP, this launch only drains
    // the few it deferred: one workgroup per CU is plenty and keeps its end cheap.
    const int64_t slots = n_wave > 0 && n_block == 0 ? ctx->num_cu : int64_t(per_cu) * ctx->num_cu;
    int64_t grid = std::min<int64_t>(P.num, slots);
    const bool need_hbm = !want_lds || tab_worst > tab_common;
    if (need_hbm) {
        a.slot_bytes = lpb::align16(tab_worst);
        if (slot_mem) {
            const int64_t fit = slot_cap / a.slot_bytes;
            if (fit < 1)
                return fail(LP_ERR_ARG, "a %lld-byte tableau slot exceeds the %lld bytes available",
                            (long long)a.slot_bytes, (long long)slot_cap);
            grid = std::min(grid, fit);
            a.scratch = slot_mem;
        } else {
            int rc = ctx->scratch.ensure(size_t(a.slot_bytes) * size_t(grid));
            if (rc != LP_OK) return rc;
            a.scratch = static_cast<char *>(ctx->scratch.p);
        }
    }
    a.queue = pc.bq;
    a.done = pc.bd;
    a.num = P.num;
    if (n_wave > 0) {
        a.ids = defer_ids;
        a.id_base = int32_t(n_block);
        a.num_dev = pc.defer;
        a.reset_extra = pc.defer;
    } else if (list_count) {
        a.ids = list_ids;
        a.id_base = 0;
        a.num_dev = list_count;
        a.reset_extra = const_cast<int32_t *>(list_count);
    } else {
        a.ids = n_block < P.num ? defer_ids : nullptr;
        a.num = n_block;
    }
    Timer t(ctx, timing, stream, bname);
    HIP_TRY(lpb::launch_simplex(fp32, nt, a, int(grid), stream));
    t.done();
    return LP_OK;
}


// ---- Workgroup-kernel launches and their tuning ------------------------------
// A batch of one LP size that the wavefront kernel cannot take is one launch,
// tuned per size bin (the cell count of its tableau).  In a batch of mixed
// sizes every LP the wavefront kernel cannot take goes to ONE persistent
// launch of the workgroup kernel whose queue hands out the most expensive LPs
// first (each LP's tableau in LDS when it fits the launch's budget, else in
// the workgroup's device-memory slot), so the launch ends on small LPs instead
// of idling between per-size launches.  Workgroup size and placement come from
// the context's tuning table (filled by the autotuner) or a heuristic.
constexpr int kBins = 4;
// Tuning-table bin of the single workgroup-kernel launch of a batch of mixed sizes.
constexpr int kMixedBin = 4;

int bin_of(int64_t m, int64_t n)
{
    const int64_t cells = (m + 1) * (n + 1);
    return cells <= 64 * 64 ? 0 : cells <= 128 * 128 ? 1 : cells <= 256 * 256 ? 2 : 3;
}

// Untuned workgroup size: 512 threads for every bin (the autotuner picked 512 in
// every bin of the 10..300 uneven batch on MI355X).
int default_threads(int) { return 512; }

// FNV-1a over the batch's shapes and the planning flags (the plan cache key).
uint64_t shape_hash(int64_t num, const int32_t *m, const int32_t *n, uint32_t flags)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix(uint64_t(num));
    mix(flags);
    for (int64_t k = 0; k < num; ++k) mix((uint64_t(uint32_t(m[k])) << 32) | uint32_t(n[k]));
    return h;
}

// Estimated work of one LP: pivots grow with m + n, each pivot touches m x n cells.
double lp_cost(int64_t m, int64_t n) { return double(m) * double(n) * double(m + n); }

struct BinLaunch {
    int m_max = 0, n_max = 0;
    int nt = 64;
    bool force_hbm = false;
    int placement = 0;  // lp_options.placement of the call (LP_PLACE_LDS lifts the budget)
};

// One persistent launch of the workgroup kernel over the work items
// 0 .. num - 1 (host-known count) or 0 .. id_base + *num_dev - 1 (device-side
// count); item t is LP ids[t] (LP t when ids is NULL).
int launch_block(lp_ctx *ctx, bool fp32, lpb::SolveArgs a, const BinLaunch &B, const int32_t *ids, int64_t num,
                 const int32_t *num_dev, int32_t id_base, int32_t *reset_extra, int64_t grid_cap, int32_t *q,
                 int32_t *d, hipStream_t stream, bool timing, const char *name)
{
    const int64_t ts = fp32 ? 4 : 8;
    const int ncol_worst = B.n_max + B.m_max;
    lpb::LdsLayout L = lpb::lds_layout(B.m_max, ncol_worst, ts, lpb::simplex_ctrl_bytes(fp32));
    const int64_t tab_common = int64_t(B.m_max + 1) * lpb::tableau_ld(B.n_max + 1, int(ts)) * ts;
    const int64_t tab_worst = int64_t(B.m_max + 1) * lpb::tableau_ld(ncol_worst + 1, int(ts)) * ts;
    int64_t lds = L.tab;
    const bool want_lds = !B.force_hbm && L.tab + tab_common <= lds_budget(ctx, B.placement);
    if (want_lds) lds = L.tab + tab_common;
    if (lds > ctx->max_lds)
        return fail(LP_ERR_ARG, "LP of %d rows x %d columns needs %lld bytes of LDS for its index arrays "
                    "(device limit %d)", B.m_max, ncol_worst, (long long)lds, ctx->max_lds);
    a.force_hbm = B.force_hbm;
    const int per_cu = lpb::simplex_blocks_per_cu(fp32, B.nt, int(lds));
    if (per_cu < 1) return fail(LP_ERR_HIP, "occupancy query failed for %d threads, %lld B LDS", B.nt, (long long)lds);
    if (!a.force_hbm) lds = lds_share(ctx, fp32, B.nt, lds, per_cu);
    a.lds_bytes = int32_t(lds);
    int64_t grid = std::min<int64_t>(num, int64_t(per_cu) * ctx->num_cu);
    if (grid_cap > 0) grid = std::min(grid, grid_cap);
    if (grid < 1) return LP_OK;
    if (!want_lds || tab_worst > tab_common) {
        a.slot_bytes = lpb::align16(tab_worst);
        int rc = ctx->scratch.ensure(size_t(a.slot_bytes) * size_t(grid));
        if (rc != LP_OK) return rc;
        a.scratch = static_cast<char *>(ctx->scratch.p);
    }
    a.queue = q;
    a.done = d;
    a.ids = ids;
    a.num = num;
    a.num_dev = num_dev;
    a.id_base = id_base;
    a.reset_extra = reset_extra;
    Timer t(ctx, timing, stream, name);
    HIP_TRY(lpb::launch_simplex(fp32, B.nt, a, int(grid), stream));
    t.done();
    return LP_OK;
}

// Trial launches of one bin's sample: every (workgroup size, placement)
// candidate is timed with events on `stream` and the fastest stored in the
// context's table.  Synchronous.  The sampled LPs' outputs are overwritten
// by the real solve that follows.
int autotune_bin(lp_ctx *ctx, bool fp32, const lpb::SolveArgs &a, BinLaunch B, int bin, const int32_t *d_sample,
                 int64_t n_sample, int32_t *q, int32_t *d, hipStream_t stream)
{
    hipEvent_t e0 = lpb::take_event(ctx), e1 = lpb::take_event(ctx);
    if (!e0 || !e1) return fail(LP_ERR_HIP, "could not create timing events");
    float best = 1e30f, best_place[2] = {1e30f, 1e30f};
    lpb::TuneEntry choice{default_threads(bin), 0}, choice_place[2] = {choice, choice};
    const int cand_nt[4] = {64, 128, 256, 512};
    // One untimed launch first (cold caches would otherwise count against the
    // first candidate), then every candidate twice, its faster time kept.
    for (int rep = -1; rep < 2; ++rep)
        for (int hbm = 0; hbm < 2; ++hbm)
            for (int nt : cand_nt) {
                if (rep < 0 && (hbm || nt != cand_nt[0])) continue;
                BinLaunch T = B;
                T.nt = nt;
                T.force_hbm = hbm != 0;
                T.placement = hbm ? LP_PLACE_HBM : LP_PLACE_LDS;  // LDS whenever the tableau fits
                HIP_TRY(hipEventRecord(e0, stream));
                int rc = launch_block(ctx, fp32, a, T, d_sample, n_sample, nullptr, 0, nullptr, 0, q, d, stream,
                                      false, "");
                if (rc != LP_OK) return rc;
                HIP_TRY(hipEventRecord(e1, stream));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (rep >= 0 && ms < best_place[hbm]) { best_place[hbm] = ms; choice_place[hbm] = lpb::TuneEntry{nt, hbm}; }
            }
    // Device-memory placement only when it wins by 5 %: the sample holds at
    // most 512 LPs, and on whole mixed batches the LDS share measured faster
    // whenever the two were within a few percent on the sample.
    const int pick = best_place[1] < 0.95f * best_place[0] ? 1 : 0;
    best = best_place[pick];
    choice = choice_place[pick];
    ctx->tune[lpb::tune_key(bin, fp32)] = choice;
    ctx->events_used -= 2;  // give the two events back to the pool
    return LP_OK;
}


struct BinSpan {
    int bin;
    int64_t offset, count;  // in the host-built id list
    int m_max, n_max;
    int64_t sample_offset, sample_count;
};

// Main pass of an uneven batch: the wavefront kernel for the LPs it fits,
// one workgroup-kernel launch per size bin (largest bin first), then one
// small launch for the LPs the wavefront kernel deferred.
int queue_binned(lp_ctx *ctx, const Plan &P, const lpb::SolveArgs &a, const lp_options &opts, PassCounters pc,
                 const int32_t *wave_ids, int64_t n_wave, int wm_max, int wn_max, int32_t *d_block,
                 int64_t n_block, const std::vector<BinSpan> &bins, const int32_t *d_samples, bool autotune,
                 hipStream_t stream, bool timing, const char *wname, const char *bname)
{
    const bool fp32 = P.fp32;
    for (const BinSpan &sp : bins) {
        if (!autotune || sp.sample_count < 1 || ctx->tune.count(lpb::tune_key(sp.bin, fp32))) continue;
        BinLaunch B;
        B.m_max = sp.m_max;
        B.n_max = sp.n_max;
        int rc = autotune_bin(ctx, fp32, a, B, sp.bin, d_samples + sp.sample_offset, sp.sample_count, pc.bq, pc.bd,
                              stream);
        if (rc != LP_OK) return rc;
    }
    if (n_wave > 0) {
        int rc = launch_wave(ctx, fp32, a, pc, wave_ids, n_wave, nullptr, wm_max, wn_max, d_block, int32_t(n_block),
                             stream, timing, wname);
        if (rc != LP_OK) return rc;
    }
    for (const BinSpan &sp : bins) {
        BinLaunch B;
        B.m_max = sp.m_max;
        B.n_max = sp.n_max;
        auto it = ctx->tune.find(lpb::tune_key(sp.bin, fp32));
        const bool tuned = it != ctx->tune.end();
        B.nt = tuned ? it->second.nt : default_threads(sp.bin);
        B.force_hbm = tuned && it->second.force_hbm != 0;
        B.placement = tuned ? (B.force_hbm ? LP_PLACE_HBM : LP_PLACE_LDS) : opts.placement;
        if (opts.placement == LP_PLACE_HBM) B.force_hbm = true;
        int rc = launch_block(ctx, fp32, a, B, d_block + sp.offset, sp.count, nullptr, 0, nullptr, 0, pc.bq, pc.bd,
                              stream, timing, bname);
        if (rc != LP_OK) return rc;
    }
    if (n_wave > 0) {
        // The deferred LPs (few, with at most 128 rows): one workgroup per CU.
        BinLaunch B;
        B.m_max = wm_max;
        B.n_max = wn_max;
        B.nt = 64;
        int rc = launch_block(ctx, fp32, a, B, d_block + n_block, n_wave, pc.defer, 0, pc.defer, ctx->num_cu,
                              pc.bq, pc.bd, stream, timing, bname);
        if (rc != LP_OK) return rc;
    }
    return LP_OK;
}

// Shapes of a batch for scaling: validated like lp_batch_solve_ex; sizes of
// A, b and c (shared: the one LP's A and b).
struct ScaleShape {
    bool uniform = true;
    int64_t sa = 0, sr = 0, sc = 0;
};

int scale_shape(int64_t num, const int32_t *m, const int32_t *n, bool shared, ScaleShape &S)
{
    for (int64_t k = 0; k < num; ++k) {
        if (m[k] < 1 || n[k] < 1)
            return fail(LP_ERR_ARG, "LP %lld has m=%d n=%d (both must be >= 1)", (long long)k, m[k], n[k]);
        if (m[k] > 1000000 || n[k] > 1000000)
            return fail(LP_ERR_ARG, "LP %lld is too large (m=%d n=%d)", (long long)k, m[k], n[k]);
        S.uniform = S.uniform && m[k] == m[0] && n[k] == n[0];
        S.sa += int64_t(m[k]) * n[k];
        S.sr += m[k];
        S.sc += n[k];
        if (S.sa > (int64_t(1) << 60)) return fail(LP_ERR_ARG, "batch size overflows");
    }
    if (shared && !S.uniform) return fail(LP_ERR_ARG, "shared = 1 needs every m[k] and every n[k] equal");
    if (shared) {
        S.sa = int64_t(m[0]) * n[0];
        S.sr = m[0];
    }
    return LP_OK;
}

int scale_batch(lp_ctx *ctx, int64_t num, const double *A, const double *b, const double *c, const int32_t *m,
                const int32_t *n, int32_t passes, bool shared, const ScaleShape &S, double *A_out,
                double *b_out, double *c_out, int32_t *rexp, int32_t *cexp, hipStream_t stream, bool timing)
{
    Timer t(ctx, timing, stream, "scale_fp64");
    if (shared) {
        // One A: its factors, then every LP's c by the column factors.
        HIP_TRY(lpb::launch_scale(1, m[0], n[0], nullptr, nullptr, nullptr, nullptr, nullptr, m, n, passes, A, b,
                                  c, A_out, b_out, nullptr, rexp, cexp, stream));
        HIP_TRY(lpb::launch_ldexp(num * n[0], c, cexp, n[0], c_out, stream));
    } else if (S.uniform) {
        HIP_TRY(lpb::launch_scale(num, m[0], n[0], nullptr, nullptr, nullptr, nullptr, nullptr, m, n, passes, A, b,
                                  c, A_out, b_out, c_out, rexp, cexp, stream));
    } else {
        const size_t bytes = size_t(num) * (2 * sizeof(int32_t) + 3 * sizeof(int64_t));
        int rc = ctx->scale_meta.ensure(bytes);
        if (rc != LP_OK) return rc;
        std::vector<char> host(bytes);
        int32_t *hm = reinterpret_cast<int32_t *>(host.data());
        int32_t *hn = hm + num;
        int64_t *ha = reinterpret_cast<int64_t *>(hn + num);
        int64_t *hr = ha + num, *hc = hr + num;
        int64_t oa = 0, orr = 0, oc = 0;
        for (int64_t k = 0; k < num; ++k) {
            hm[k] = m[k]; hn[k] = n[k];
            ha[k] = oa; hr[k] = orr; hc[k] = oc;
            oa += int64_t(m[k]) * n[k]; orr += m[k]; oc += n[k];
        }
        HIP_TRY(hipMemcpyAsync(ctx->scale_meta.p, host.data(), bytes, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));  // the host staging buffer goes away
        const int32_t *dm = ctx->scale_meta.as<int32_t>();
        const int64_t *da = reinterpret_cast<const int64_t *>(dm + 2 * num);
        HIP_TRY(lpb::launch_scale(num, 0, 0, dm, dm + num, da, da + num, da + 2 * num, m, n, passes, A, b, c,
                                  A_out, b_out, c_out, rexp, cexp, stream));
    }
    t.done();
    return LP_OK;
}

// lp_batch_solve_ex with opts.scaling > 0: scale into context scratch, solve
// the scaled batch, map x back (x_j = x'_j 2^s_j; obj and status carry over).
int solve_scaled(lp_ctx *ctx, int64_t num, const double *A, const double *b, const double *c, const int8_t *sense,
                 const int32_t *m, const int32_t *n, int32_t *status, double *x, double *obj,
                 const lp_options &opts)
{
    const bool shared = opts.shared != 0;
    ScaleShape S;
    int rc = scale_shape(num, m, n, shared, S);
    if (rc != LP_OK) return rc;
    const int64_t nc = shared ? num * int64_t(n[0]) : S.sc;
    const size_t oA = 0, ob = oA + lpb::align16(8 * size_t(S.sa)), oc = ob + lpb::align16(8 * size_t(S.sr)),
                 orx = oc + lpb::align16(8 * size_t(nc)), ocx = orx + lpb::align16(4 * size_t(S.sr)),
                 end = ocx + lpb::align16(4 * size_t(S.sc));
    rc = ctx->scaled.ensure(end);
    if (rc != LP_OK) return rc;
    double *As = ctx->scaled.as<double>(oA), *bs = ctx->scaled.as<double>(ob), *cs = ctx->scaled.as<double>(oc);
    int32_t *rx = ctx->scaled.as<int32_t>(orx), *cx = ctx->scaled.as<int32_t>(ocx);
    hipStream_t stream = reinterpret_cast<hipStream_t>(opts.stream);
    const bool timing = (opts.flags & LP_FLAG_TIME_KERNELS) != 0;
    rc = scale_batch(ctx, num, A, b, c, m, n, opts.scaling, shared, S, As, bs, cs, rx, cx, stream, timing);
    if (rc != LP_OK) return rc;
    lp_options o = opts;
    o.scaling = 0;
    o.flags &= ~LP_FLAG_SYNC;
    rc = lp_batch_solve_ex(ctx, num, As, bs, cs, sense, m, n, status, x, obj, &o);
    if (rc != LP_OK) return rc;
    {
        Timer t(ctx, timing, stream, "unscale_x");
        HIP_TRY(lpb::launch_ldexp(nc, x, cx, shared ? n[0] : 0, x, stream));
        t.done();
    }
    if (opts.flags & LP_FLAG_SYNC) HIP_TRY(hipStreamSynchronize(stream));
    return LP_OK;
}

}  // namespace

extern "C" {

const char *lp_last_error(void) { return lpb::g_last_error.c_str(); }

void lp_options_init(lp_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->precision = LP_PREC_FP64;
    o->k_deg = 50;
}

int lp_ctx_create(lp_ctx **out, int device)
{
    if (!out) return fail(LP_ERR_ARG, "lp_ctx_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(LP_ERR_ARG, "lp_ctx_create: device %d out of range (%d devices)", device, ndev);
    DeviceGuard g(device);
    lp_ctx *ctx = new lp_ctx;
    ctx->device = device;
    hipError_t e1 = hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, device);
    hipError_t e2 = hipDeviceGetAttribute(&ctx->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (hipDeviceGetAttribute(&ctx->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) !=
            hipSuccess ||
        ctx->lds_per_cu < ctx->max_lds)
        ctx->lds_per_cu = ctx->max_lds;
    if (e1 != hipSuccess || e2 != hipSuccess) {
        delete ctx;
        return fail(LP_ERR_HIP, "lp_ctx_create: device attribute query failed");
    }
    if (lpb::simplex_configure(ctx->max_lds) != hipSuccess ||
        lpb::simplex_wave_configure(ctx->max_lds) != hipSuccess ||
        lpb::certify_configure(ctx->max_lds) != hipSuccess || lpb::certify_dense_configure(ctx->max_lds) != hipSuccess ||
        lpb::mlp_configure() != hipSuccess) {
        delete ctx;
        return fail(LP_ERR_HIP, "lp_ctx_create: could not configure kernel LDS limits");
    }
    // This device's copy of the no-allocation entry point's static scratch:
    // its device address, looked up with the device current (the array's
    // host-side name is not a device address).  A failure only disables
    // lp_batch_solve_noalloc, which then reports it.
    ctx->noalloc_err = int(lpb::noalloc_scratch_address(&ctx->noalloc));
    if (ctx->noalloc_err != hipSuccess) ctx->noalloc = nullptr;
    int rc = ctx->counters.ensure(4096);
    if (rc == LP_OK && (lpb::launch_zero_i32(static_cast<int32_t *>(ctx->counters.p), 1024, nullptr) != hipSuccess ||
                        hipStreamSynchronize(nullptr) != hipSuccess))
        rc = fail(LP_ERR_HIP, "lp_ctx_create: could not clear the work counters");
    if (rc != LP_OK) {
        delete ctx;
        return rc;
    }
    *out = ctx;
    return LP_OK;
}

void lp_ctx_destroy(lp_ctx *ctx)
{
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->scratch.release();
    ctx->meta.release();
    ctx->scaled.release();
    ctx->scale_meta.release();
    ctx->counters.release();
    lpb::MlpState &M = ctx->mlp;
    for (lpb::DevBuf *d : {&M.params, &M.params16, &M.adam_m, &M.adam_v, &M.grads, &M.act, &M.misc})
        d->release();
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    lpb::HostPipe &H = ctx->pipe;
    for (lpb::PipeSet &S : H.set) {
        S.dev.release();
        S.in.release();
        S.out.release();
        for (hipEvent_t e : {S.up, S.solved, S.down})
            if (e) (void)hipEventDestroy(e);
    }
    for (hipStream_t st : {H.h2d, H.comp, H.d2h})
        if (st) (void)hipStreamDestroy(st);
    ctx->plan.staging.release();
    if (ctx->plan.uploaded) (void)hipEventDestroy(ctx->plan.uploaded);
    delete ctx;
}

int lp_batch_solve_ex(lp_ctx *ctx, int64_t num_lps, const double *A, const double *b,
                      const double *c, const int8_t *sense, const int32_t *m, const int32_t *n,
                      int32_t *status, double *x, double *obj, const lp_options *opts_in)
{
    if (!ctx) return fail(LP_ERR_ARG, "lp_batch_solve_ex: ctx is NULL");
    if (num_lps < 0) return fail(LP_ERR_ARG, "num_lps is negative (%lld)", (long long)num_lps);
    lp_options opts;
    lp_options_init(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.precision != LP_PREC_FP64 && opts.precision != LP_PREC_FP32_CERT64)
        return fail(LP_ERR_ARG, "unknown precision %d", opts.precision);
    if (opts.block_threads && opts.block_threads != 64 && opts.block_threads != 128 &&
        opts.block_threads != 256 && opts.block_threads != 512)
        return fail(LP_ERR_ARG, "block_threads must be 0, 64, 128, 256 or 512");
    if (opts.placement < 0 || opts.placement > LP_PLACE_HBM)
        return fail(LP_ERR_ARG, "unknown placement %d", opts.placement);
    if (opts.scaling < 0 || opts.scaling > 64) return fail(LP_ERR_ARG, "scaling must lie in 0..64 (got %d)", opts.scaling);
    if (opts.pricing != LP_PRICE_DANTZIG && opts.pricing != LP_PRICE_STEEPEST_EDGE)
        return fail(LP_ERR_ARG, "unknown pricing %d", opts.pricing);
    if (num_lps == 0) return LP_OK;
    if (!A || !b || !c || !sense || !m || !n || !status || !x || !obj)
        return fail(LP_ERR_ARG, "a batch pointer is NULL");
    if (num_lps > INT32_MAX) return fail(LP_ERR_ARG, "num_lps exceeds 2^31-1");
    if (opts.scaling > 0) {
        DeviceGuard g(ctx->device);
        return solve_scaled(ctx, num_lps, A, b, c, sense, m, n, status, x, obj, opts);
    }

    // Shapes (host arrays) and the uniform-shape shortcut.
    Plan P;
    P.num = num_lps;
    P.m0 = m[0]; P.n0 = n[0]; P.m_max = 0; P.n_max = 0; P.mn_max = 0;
    P.uniform = true;
    int64_t sa = 0;
    for (int64_t k = 0; k < num_lps; ++k) {
        const int32_t mk = m[k], nk = n[k];
        if (mk < 1 || nk < 1)
            return fail(LP_ERR_ARG, "LP %lld has m=%d n=%d (both must be >= 1)", (long long)k, mk, nk);
        if (mk > 1000000 || nk > 1000000)
            return fail(LP_ERR_ARG, "LP %lld is too large (m=%d n=%d)", (long long)k, mk, nk);
        P.uniform = P.uniform && mk == P.m0 && nk == P.n0;
        P.m_max = std::max(P.m_max, mk);
        P.n_max = std::max(P.n_max, nk);
        P.mn_max = std::max<int64_t>(P.mn_max, int64_t(mk) * nk);
        sa += int64_t(mk) * nk;
        if (sa > (int64_t(1) << 60)) return fail(LP_ERR_ARG, "batch size overflows");
    }
    P.fp32 = opts.precision == LP_PREC_FP32_CERT64;
    P.ts = P.fp32 ? 4 : 8;
    // Shared constraints, optionally screened: the first pass solves every LP
    // on its subset_m rows only, and the certificate judges the basis on all rows.
    const bool shared = opts.shared != 0;
    const bool screened = opts.row_subset != nullptr;
    if (screened && !shared) return fail(LP_ERR_ARG, "row_subset needs shared = 1");
    if (shared && !P.uniform) return fail(LP_ERR_ARG, "shared = 1 needs every m[k] and every n[k] equal");
    if (screened && (opts.subset_m < 1 || opts.subset_m > P.m0))
        return fail(LP_ERR_ARG, "subset_m = %d must lie in 1..%d", opts.subset_m, P.m0);
    const Plan P_full = P;
    if (screened) P.m0 = P.m_max = opts.subset_m;
    const bool certify = P.fp32 || screened;
    hipStream_t stream = reinterpret_cast<hipStream_t>(opts.stream);
    DeviceGuard g(ctx->device);

    // Kernel choice per LP: one wavefront for LPs of at most 64 columns and 128
    // rows whose tableau fits LDS, a workgroup otherwise (or when the caller
    // fixes the workgroup size or asks for HBM placement).
    const bool auto_kernel = opts.block_threads == 0 && opts.placement != LP_PLACE_HBM;
    std::vector<int32_t> wave_ids, block_ids;
    int64_t n_wave = 0, rows = 0;
    int wm_max = 0, wn_max = 0;
    if (P.uniform) {
        const bool w = auto_kernel && wave_fit(ctx, P.m0, P.n0, P.fp32, screened);
        n_wave = w ? num_lps : 0;
        wm_max = w ? P.m0 : 0;
        wn_max = w ? P.n0 : 0;
        rows = num_lps * int64_t(P.m0);
    } else {
        for (int64_t k = 0; k < num_lps; ++k) {
            const bool w = auto_kernel && wave_fit(ctx, m[k], n[k], P.fp32, false);
            if (w) {
                ++n_wave;
                wm_max = std::max(wm_max, m[k]);
                wn_max = std::max(wn_max, n[k]);
            }
            rows += m[k];
            (w ? wave_ids : block_ids).push_back(int32_t(k));
        }
    }
    const int64_t n_block = num_lps - n_wave;

    lpb::SolveArgs a;
    std::memset(&a, 0, sizeof a);
    a.A = A; a.b = b; a.c = c; a.sense = sense;
    a.status = status; a.x = x; a.obj = obj;
    a.stats = opts.stats;
    a.prm = fill_params(opts, P.fp32);
    a.shared = shared ? 1 : 0;
    a.row_subset = opts.row_subset;
    a.m_full = P_full.m0;

    // Device metadata: [m][n][aoff][roff][coff] (non-uniform only); id lists
    // (capacity num_lps each): wavefront ids, deferred/workgroup ids, fallback
    // ids, deferred ids of the fallback pass; FP32 final bases [rows] and
    // entering variables [num_lps].
    const size_t sz_shape = P.uniform ? 0 : size_t(num_lps) * (2 * sizeof(int32_t) + 3 * sizeof(int64_t));
    const size_t sz_ids = size_t(num_lps) * sizeof(int32_t);
    const size_t sz_fp32 = certify ? lpb::align16(size_t(rows) * 4) + 2 * lpb::align16(sz_ids) : 0;
    {
        int rc = ctx->meta.ensure(sz_shape + 4 * lpb::align16(sz_ids) + sz_fp32);
        if (rc != LP_OK) return rc;
        // A batch of one size writes id lists where a mixed batch's plan lives.
        if (P.uniform) ctx->plan.valid = false;
    }
    char *meta = static_cast<char *>(ctx->meta.p);
    int32_t *d_wave_ids = reinterpret_cast<int32_t *>(meta + sz_shape);
    int32_t *d_defer_ids = reinterpret_cast<int32_t *>(meta + sz_shape + lpb::align16(sz_ids));
    int32_t *d_fb_ids = reinterpret_cast<int32_t *>(meta + sz_shape + 2 * lpb::align16(sz_ids));
    int32_t *d_fb_defer = reinterpret_cast<int32_t *>(meta + sz_shape + 3 * lpb::align16(sz_ids));
    int32_t *d_basis = reinterpret_cast<int32_t *>(meta + sz_shape + 4 * lpb::align16(sz_ids));
    int32_t *d_enter = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(d_basis) + lpb::align16(size_t(rows) * 4));
    int32_t *d_viol = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(d_enter) + lpb::align16(sz_ids));
    // Uneven batches with automatic kernel choice: size bins for the LPs the
    // wavefront kernel cannot take, each bin ordered by estimated work
    // (largest first), bins largest first; plus a sample of every bin for the
    // autotuner.
    // A uniform batch the workgroup kernel takes is a single bin, binned when
    // it is tuned or to be tuned.
    const bool autotune = (opts.flags & LP_FLAG_AUTOTUNE) != 0;
    const bool binned = auto_kernel && n_block > 0 &&
                        (!P.uniform || autotune || ctx->tune.count(lpb::tune_key(bin_of(P.m0, P.n0), P.fp32)));
    std::vector<BinSpan> bins;
    std::vector<int32_t> samples;
    if (binned && P.uniform) {
        BinSpan sp;
        sp.bin = bin_of(P.m0, P.n0);
        sp.offset = 0;
        sp.count = num_lps;
        sp.m_max = P.m0;
        sp.n_max = P.n0;
        sp.sample_offset = 0;
        sp.sample_count = std::min<int64_t>(num_lps, 512);
        for (int64_t t = 0; t < sp.sample_count; ++t) samples.push_back(int32_t(t * num_lps / sp.sample_count));
        bins.push_back(sp);
    } else if (binned) {
        // Every LP the wavefront kernel cannot take, in one launch, ordered by
        // estimated work (largest first); the autotuner's sample is every
        // stride-th LP of that order, at most 512.
        std::stable_sort(block_ids.begin(), block_ids.end(),
                         [&](int32_t x, int32_t y) { return lp_cost(m[x], n[x]) > lp_cost(m[y], n[y]); });
        BinSpan sp;
        sp.bin = kMixedBin;
        sp.offset = 0;
        sp.count = int64_t(block_ids.size());
        sp.m_max = 0;
        sp.n_max = 0;
        for (int32_t k : block_ids) { sp.m_max = std::max(sp.m_max, m[k]); sp.n_max = std::max(sp.n_max, n[k]); }
        sp.sample_offset = 0;
        const int64_t want = std::min<int64_t>(sp.count, 512);
        for (int64_t t = 0; t < want; ++t) samples.push_back(block_ids[size_t(t * sp.count / want)]);
        sp.sample_count = want;
        bins.push_back(sp);
    }
    if (P.uniform) {
        a.um = P.m0;
        a.un = P.n0;
        if (autotune && !samples.empty()) {
            HIP_TRY(hipMemcpyAsync(d_fb_defer, samples.data(), samples.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, stream));
            HIP_TRY(hipStreamSynchronize(stream));
        }
    } else {
        // Shapes, offsets and id lists of a batch of mixed sizes: reused from
        // the previous call when it planned the same shapes (nothing to upload,
        // so repeat solves can be captured in a HIP graph); otherwise uploaded
        // from the context's pinned staging buffer without waiting for the copy.
        const bool need_samples = autotune && !bins.empty() && !ctx->tune.count(lpb::tune_key(kMixedBin, P.fp32));
        const uint32_t plan_flags = (P.fp32 ? 1u : 0u) | (auto_kernel ? 2u : 0u) | (binned ? 4u : 0u);
        const uint64_t h = shape_hash(num_lps, m, n, plan_flags);
        const bool hit = ctx->plan.valid && ctx->plan.hash == h && ctx->plan.meta_p == ctx->meta.p &&
                         ctx->plan.meta_bytes == ctx->meta.bytes && !need_samples;
        if (!hit) {
            hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
            HIP_TRY(hipStreamIsCapturing(stream, &cap));
            if (cap != hipStreamCaptureStatusNone)
                return fail(LP_ERR_ARG, "a batch of mixed LP sizes can be captured in a graph only after an "
                            "uncaptured solve of the same shapes on this context (its plan is then reused)");
            const size_t sample_at = sz_shape + 3 * lpb::align16(sz_ids);
            const size_t bytes = samples.empty() ? sz_shape + lpb::align16(sz_ids) + size_t(n_block) * sizeof(int32_t)
                                                 : sample_at + samples.size() * sizeof(int32_t);
            // The previous upload must have read the staging buffer before it is rewritten.
            if (ctx->plan.uploaded) HIP_TRY(hipEventSynchronize(ctx->plan.uploaded));
            else HIP_TRY(hipEventCreateWithFlags(&ctx->plan.uploaded, hipEventDisableTiming));
            ctx->plan.valid = false;
            int rc = ctx->plan.staging.ensure(bytes);
            if (rc != LP_OK) return rc;
            char *host = static_cast<char *>(ctx->plan.staging.p);
            if (!samples.empty()) std::copy(samples.begin(), samples.end(), reinterpret_cast<int32_t *>(host + sample_at));
            int32_t *hm = reinterpret_cast<int32_t *>(host);
            int32_t *hn = hm + num_lps;
            int64_t *ha = reinterpret_cast<int64_t *>(hn + num_lps);
            int64_t *hr = ha + num_lps, *hc = hr + num_lps;
            int64_t oa = 0, orr = 0, oc = 0;
            for (int64_t k = 0; k < num_lps; ++k) {
                hm[k] = m[k]; hn[k] = n[k];
                ha[k] = oa; hr[k] = orr; hc[k] = oc;
                oa += int64_t(m[k]) * n[k]; orr += m[k]; oc += n[k];
            }
            int32_t *hw = reinterpret_cast<int32_t *>(host + sz_shape);
            std::copy(wave_ids.begin(), wave_ids.end(), hw);
            int32_t *hb = reinterpret_cast<int32_t *>(host + sz_shape + lpb::align16(sz_ids));
            std::copy(block_ids.begin(), block_ids.end(), hb);
            HIP_TRY(hipMemcpyAsync(meta, host, bytes, hipMemcpyHostToDevice, stream));
            HIP_TRY(hipEventRecord(ctx->plan.uploaded, stream));
            ctx->plan.valid = true;
            ctx->plan.hash = h;
            ctx->plan.meta_p = ctx->meta.p;
            ctx->plan.meta_bytes = ctx->meta.bytes;
        }
        a.m = reinterpret_cast<int32_t *>(meta);
        a.n = a.m + num_lps;
        a.aoff = reinterpret_cast<int64_t *>(const_cast<int32_t *>(a.n + num_lps));
        a.roff = a.aoff + num_lps;
        a.coff = a.roff + num_lps;
    }
    // Work counters, each returned to 0 by the last workgroup of its launch.
    int32_t *cnt = static_cast<int32_t *>(ctx->counters.p);
    PassCounters main_pc{cnt + 0, cnt + 1, cnt + 2, cnt + 3, cnt + 4};
    PassCounters fb_pc{cnt + 16, cnt + 17, cnt + 18, cnt + 19, cnt + 20};
    int32_t *cert_q = cnt + 8, *cert_d = cnt + 9, *fb_count = cnt + 10;
    const bool timing = (opts.flags & LP_FLAG_TIME_KERNELS) != 0;
    if (ctx->counters_dirty) {
        HIP_TRY(lpb::launch_zero_i32(cnt, 1024, stream));
        ctx->counters_dirty = false;
    }
    ctx->counters_dirty = true;  // until every launch below has been queued

    if (certify) {
        a.basis_out = d_basis;
        a.enter_out = d_enter;
    }
    const char *wname = screened ? (P.fp32 ? "simplex_wave_fp32_screened" : "simplex_wave_fp64_screened")
                                 : (P.fp32 ? "simplex_wave_fp32" : "simplex_wave_fp64");
    const char *bname = screened ? (P.fp32 ? "simplex_block_fp32_screened" : "simplex_block_fp64_screened")
                                 : (P.fp32 ? "simplex_block_fp32" : "simplex_block_fp64");
    int rc = binned ? queue_binned(ctx, P, a, opts, main_pc, d_wave_ids, n_wave, wm_max, wn_max,
                                   P.uniform ? nullptr : d_defer_ids, n_block, bins, d_fb_defer, autotune, stream,
                                   timing, wname, bname)
                    : queue_pass(ctx, P, a, opts, main_pc, P.uniform ? nullptr : d_wave_ids, n_wave, wm_max,
                                 wn_max, n_block, d_defer_ids, nullptr, nullptr, stream, timing, wname, bname);
    if (rc != LP_OK) return rc;

    if (certify) {
        // FP64 certificate of every final basis, then an FP64 re-solve of the rest.
        lpb::CertArgs ca;
        std::memset(&ca, 0, sizeof ca);
        ca.num = num_lps;
        ca.A = A; ca.b = b; ca.c = c; ca.sense = sense;
        ca.um = P_full.uniform ? P_full.m0 : 0; ca.un = a.un; ca.m = a.m; ca.n = a.n;
        ca.shared = a.shared;
        ca.row_subset = opts.row_subset;
        ca.subset_m = screened ? opts.subset_m : 0;
        ca.aoff = a.aoff; ca.roff = a.roff; ca.coff = a.coff;
        ca.status = status; ca.x = x; ca.obj = obj; ca.stats = opts.stats;
        ca.basis = d_basis; ca.enter = d_enter;
        ca.fb_ids = d_fb_ids; ca.fb_count = fb_count;
        ca.viol = nullptr;
        bool viol_counted = false;
        ca.queue = cert_q; ca.done = cert_d;
        const lpb::SolveParams p64 = fill_params(opts, false);
        ca.tol_feas = p64.tol_feas;
        ca.tol_opt = p64.tol_opt;
        const int kmax = std::min(P_full.m_max, P_full.n_max);
        const bool dense = !shared && P_full.m_max <= 64 && P_full.n_max <= 64 &&
                           P_full.mn_max <= lpb::certify_dense_prefetch_elems();
        if (dense) {
            // One wavefront per LP with the next LP's input in flight; LU blocks
            // up to 20 x 20 (a larger basis goes to the FP64 re-solve).
            const int kl = std::min(kmax, 20);
            const int64_t lds = lpb::certify_dense_lds_bytes(P_full.m_max, P_full.n_max, kl);
            if (lds > ctx->max_lds) return fail(LP_ERR_ARG, "LP too large for the certificate kernel");
            ca.wave_bytes = int32_t(lpb::certify_dense_a_bytes(P_full.m_max, P_full.n_max));
            ca.kl = kl;
            ca.lds_bytes = int32_t(lds);
            ca.viol = d_viol;
            viol_counted = true;
            const int per_cu = lpb::certify_dense_blocks_per_cu(int(lds));
            if (per_cu < 1) return fail(LP_ERR_HIP, "occupancy query failed for the certificate kernel");
            const int64_t cgrid = std::min<int64_t>(num_lps, int64_t(per_cu) * ctx->num_cu);
            Timer t(ctx, timing, stream, "certify_fp64");
            HIP_TRY(lpb::launch_certify_dense(ca, int(cgrid), stream));
            t.done();
        } else if (kmax <= 64) {
            // One wavefront per LP; LU blocks up to kl x kl in LDS (a basis with
            // more basic structurals, rare at these sizes, goes to the FP64
            // re-solve).  Shared constraints are copied into LDS once per
            // workgroup of W wavefronts when they fit next to W wavefront regions.
            const int64_t a_bytes = lpb::align16(8 * int64_t(P_full.m0) * (P_full.n0 | 1));  // rows at an odd stride
            int W = 1, kl = std::min(kmax, 32), stage = 0;
            int64_t wb = lpb::wave_cert_layout(P_full.m_max, P_full.n_max, kl).end, lds = wb;
            if (shared && a_bytes <= 65536) {
                const int cand_w[4] = {16, 16, 8, 8};
                const int cand_k[4] = {32, 24, 32, 24};
                for (int q = 0; q < 4 && !stage; ++q) {
                    const int klq = std::min(kmax, cand_k[q]);
                    const int64_t wbq = lpb::wave_cert_layout(P_full.m_max, P_full.n_max, klq).end;
                    if (a_bytes + cand_w[q] * wbq <= ctx->max_lds) {
                        W = cand_w[q]; kl = klq; wb = wbq; lds = a_bytes + W * wbq; stage = 1;
                    }
                }
            }
            if (lds > ctx->max_lds) return fail(LP_ERR_ARG, "LP too large for the certificate kernel");
            ca.wave_bytes = int32_t(wb);
            ca.kl = kl;
            ca.stage_a = stage;
            ca.lds_bytes = int32_t(lds);
            ca.viol = d_viol;
            viol_counted = true;
            const int per_cu = lpb::certify_wave_blocks_per_cu(W, int(lds));
            if (per_cu < 1) return fail(LP_ERR_HIP, "occupancy query failed for the certificate kernel");
            const int64_t cgrid = std::min<int64_t>((num_lps + W - 1) / W, int64_t(per_cu) * ctx->num_cu);
            Timer t(ctx, timing, stream, "certify_fp64");
            HIP_TRY(lpb::launch_certify_wave(W, ca, int(cgrid), stream));
            t.done();
        } else {
            // One workgroup of 64 threads per LP; LU blocks up to 32 x 32 in LDS,
            // larger ones in the workgroup's device-memory slot.
            const int cnt_nt = 64;
            const int64_t kl = std::min(kmax, 32);
            const int64_t clds = lpb::certify_lds_bytes(P_full.m_max, P_full.n_max, false) + 8 * kl * kl;
            if (clds > ctx->max_lds) return fail(LP_ERR_ARG, "LP too large for the certificate kernel");
            ca.lds_bytes = int32_t(clds);
            const int per_cu = lpb::certify_blocks_per_cu(cnt_nt, int(clds));
            if (per_cu < 1) return fail(LP_ERR_HIP, "occupancy query failed for the certificate kernel");
            const int64_t cgrid = std::min<int64_t>(num_lps, int64_t(per_cu) * ctx->num_cu);
            ca.slot_bytes = lpb::align16(8 * int64_t(kmax) * kmax);
            if (!P.uniform && n_block + n_wave == num_lps) {
                // The workgroup kernel's LPs in its order (largest first), then the rest.
                ca.order1 = d_defer_ids;
                ca.n1 = n_block;
                ca.order2 = d_wave_ids;
            }
            int rc2 = ctx->scratch.ensure(std::max<size_t>(ctx->scratch.bytes, size_t(ca.slot_bytes) * size_t(cgrid)));
            if (rc2 != LP_OK) return rc2;
            ca.scratch = static_cast<char *>(ctx->scratch.p);
            Timer t(ctx, timing, stream, "certify_fp64");
            HIP_TRY(lpb::launch_certify(cnt_nt, ca, int(cgrid), stream));
            t.done();
        }
        // FP64 re-solve of every LP the certificate rejected, on all of its rows.
        Plan P64 = P_full;
        P64.fp32 = false;
        P64.ts = 8;
        lpb::SolveArgs a64 = a;
        a64.prm = fill_params(opts, false);
        a64.basis_out = nullptr;
        a64.enter_out = nullptr;
        a64.refine_stats = 1;
        a64.row_subset = nullptr;
        // Start each re-solve from the single-precision solve's final basis --
        // of the relaxation when screened, of the LP itself otherwise -- and
        // repair it with the dual (or primal) simplex method; LPs the repair
        // does not finish go on to a solve from the slack basis.
        a64.warm_basis = d_basis;
        a64.warm_rows = screened ? opts.row_subset : nullptr;
        a64.warm_m = screened ? opts.subset_m : 0;
        // A start whose x violates many rows is far from the LP's optimum: the
        // slack-basis solve is cheaper than the repair then.
        a64.warm_viol = viol_counted ? d_viol : nullptr;
        a64.warm_max_viol = 16;
        if (P_full.uniform) a64.um = P_full.m0;
        int64_t n_wave64 = 0;
        int wm64 = 0, wn64 = 0;
        if (P_full.uniform) {
            if (auto_kernel && wave_fit(ctx, P_full.m0, P_full.n0, false, false)) {
                n_wave64 = num_lps;
                wm64 = P_full.m0;
                wn64 = P_full.n0;
            }
        } else {
            for (int64_t k = 0; k < num_lps && auto_kernel; ++k)
                if (wave_fit(ctx, m[k], n[k], false, false)) {
                    ++n_wave64;
                    wm64 = std::max(wm64, m[k]);
                    wn64 = std::max(wn64, n[k]);
                }
        }
        rc = queue_pass(ctx, P64, a64, opts, fb_pc, nullptr, n_wave64 > 0 ? 1 : 0, wm64, wn64, 0, d_fb_defer,
                        d_fb_ids, fb_count, stream, timing, "simplex_wave_fp64_resolve",
                        "simplex_block_fp64_resolve");
        if (rc != LP_OK) return rc;
    }
    ctx->counters_dirty = false;
    if (opts.flags & LP_FLAG_SYNC) HIP_TRY(hipStreamSynchronize(stream));
    return LP_OK;
}

int lp_batch_solve_noalloc(lp_ctx *ctx, int64_t num_lps, const double *A, const double *b, const double *c,
                           const int8_t *sense, int32_t m, int32_t n, int32_t *status, double *x, double *obj,
                           int32_t *stats, void *stream_p)
{
    if (!ctx) return fail(LP_ERR_ARG, "lp_batch_solve_noalloc: ctx is NULL");
    if (num_lps < 0 || num_lps > lpb::kNoAllocMaxLps)
        return fail(LP_ERR_ARG, "lp_batch_solve_noalloc: num_lps = %lld outside 0..%lld", (long long)num_lps,
                    (long long)lpb::kNoAllocMaxLps);
    if (num_lps == 0) return LP_OK;
    if (!A || !b || !c || !sense || !status || !x || !obj)
        return fail(LP_ERR_ARG, "lp_batch_solve_noalloc: a batch pointer is NULL");
    if (m < 1 || n < 1) return fail(LP_ERR_ARG, "lp_batch_solve_noalloc: m = %d, n = %d (both must be >= 1)", m, n);
    if (!wave_fit(ctx, m, n, false, false))
        return fail(LP_ERR_ARG, "lp_batch_solve_noalloc: LPs of %d x %d exceed one wavefront's tableau "
                    "(at most 64 columns and 128 rows, in LDS)", m, n);
    if (!ctx->noalloc)
        return fail(LP_ERR_HIP, "lp_batch_solve_noalloc: no device address for the static scratch (%s)",
                    hipGetErrorString(hipError_t(ctx->noalloc_err)));
    // A deferred LP (more columns than the wavefront holds once >= rows add
    // their surplus columns) needs one workgroup-kernel slot at least.
    const int64_t slot = lpb::align16(int64_t(m + 1) * lpb::tableau_ld(n + m + 1, 8) * 8);
    if (slot > lpb::kNoAllocBytes - lpb::kNoAllocSlotsAt)
        return fail(LP_ERR_ARG, "lp_batch_solve_noalloc: LPs of %d x %d need a larger tableau slot", m, n);
    DeviceGuard g(ctx->device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_p);

    Plan P;
    P.num = num_lps;
    P.uniform = true;
    P.m0 = P.m_max = m;
    P.n0 = P.n_max = n;
    P.mn_max = int64_t(m) * n;
    P.fp32 = false;
    P.ts = 8;
    lp_options opts;
    lp_options_init(&opts);
    lpb::SolveArgs a;
    std::memset(&a, 0, sizeof a);
    a.A = A; a.b = b; a.c = c; a.sense = sense;
    a.status = status; a.x = x; a.obj = obj;
    a.stats = stats;
    a.prm = fill_params(opts, false);
    a.um = m;
    a.un = n;
    // Scratch: the counters start at zero (cleared here by a kernel; every
    // launch returns its counters to zero when it ends).
    char *base = static_cast<char *>(ctx->noalloc);
    int32_t *cnt = reinterpret_cast<int32_t *>(base);
    HIP_TRY(lpb::launch_zero_i32(cnt, 64, stream));
    PassCounters pc{cnt + 0, cnt + 1, cnt + 2, cnt + 3, cnt + 4};
    int32_t *defer_ids = reinterpret_cast<int32_t *>(base + lpb::kNoAllocIdsAt);
    return queue_pass(ctx, P, a, opts, pc, nullptr, num_lps, m, n, 0, defer_ids, nullptr, nullptr, stream, false,
                      "", "", base + lpb::kNoAllocSlotsAt, lpb::kNoAllocBytes - lpb::kNoAllocSlotsAt);
}

int lp_batch_scale(lp_ctx *ctx, int64_t num_lps, const double *A, const double *b, const double *c,
                   const int32_t *m, const int32_t *n, int32_t passes, int32_t shared, double *A_out,
                   double *b_out, double *c_out, int32_t *row_exp, int32_t *col_exp, void *stream)
{
    if (!ctx) return fail(LP_ERR_ARG, "lp_batch_scale: ctx is NULL");
    if (num_lps < 0) return fail(LP_ERR_ARG, "num_lps is negative (%lld)", (long long)num_lps);
    if (passes < 0 || passes > 64) return fail(LP_ERR_ARG, "passes must lie in 0..64 (got %d)", passes);
    if (num_lps == 0) return LP_OK;
    if (!A || !b || !c || !m || !n || !A_out || !b_out || !c_out || !row_exp || !col_exp)
        return fail(LP_ERR_ARG, "lp_batch_scale: a pointer is NULL");
    ScaleShape S;
    int rc = scale_shape(num_lps, m, n, shared != 0, S);
    if (rc != LP_OK) return rc;
    DeviceGuard g(ctx->device);
    return scale_batch(ctx, num_lps, A, b, c, m, n, passes, shared != 0, S, A_out, b_out, c_out, row_exp, col_exp,
                       reinterpret_cast<hipStream_t>(stream), false);
}

int lp_hyperbox_support(lp_ctx *ctx, int64_t num, int32_t n, const double *lo, const double *hi,
                        const double *l, int32_t shared_box, double *value, double *x, void *stream)
{
    if (!ctx) return fail(LP_ERR_ARG, "ctx is NULL");
    if (num < 0) return fail(LP_ERR_ARG, "num is negative (%lld)", (long long)num);
    if (n < 1 || n > 1000000) return fail(LP_ERR_ARG, "n = %d must lie in 1..1000000", n);
    if (num == 0) return LP_OK;
    if (!lo || !hi || !l || !value) return fail(LP_ERR_ARG, "a box pointer is NULL");
    if (num > (int64_t(1) << 40) / n) return fail(LP_ERR_ARG, "batch size overflows");
    DeviceGuard g(ctx->device);
    HIP_TRY(lpb::launch_hyperbox(num, n, lo, hi, l, shared_box ? 1 : 0, value, x,
                                 static_cast<hipStream_t>(stream)));
    return LP_OK;
}

int lp_ctx_tuning(lp_ctx *ctx, int32_t *entries, int cap)
{
    if (!ctx) return fail(LP_ERR_ARG, "lp_ctx_tuning: ctx is NULL");
    int i = 0;
    for (const auto &kv : ctx->tune) {
        if (entries && i < cap) {
            entries[4 * i + 0] = kv.first / 2;
            entries[4 * i + 1] = kv.first % 2;
            entries[4 * i + 2] = kv.second.nt;
            entries[4 * i + 3] = kv.second.force_hbm;
        }
        ++i;
    }
    return i;
}

int lp_ctx_kernel_times(lp_ctx *ctx, const char **names, float *ms, int cap)
{
    if (!ctx) return fail(LP_ERR_ARG, "lp_ctx_kernel_times: ctx is NULL");
    DeviceGuard g(ctx->device);
    const int cnt = int(ctx->times.size());
    for (int i = 0; i < cnt && i < cap; ++i) {
        HIP_TRY(hipEventSynchronize(ctx->times[i].stop));
        float v = 0.f;
        HIP_TRY(hipEventElapsedTime(&v, ctx->times[i].start, ctx->times[i].stop));
        if (names) names[i] = ctx->times[i].name;
        if (ms) ms[i] = v;
    }
    ctx->times.clear();
    ctx->events_used = 0;
    return cnt;
}

int lp_batch_solve(int64_t num_lps, const double *A, const double *b, const double *c,
                   const int8_t *sense, const int32_t *m, const int32_t *n, int32_t *status,
                   double *x, double *obj)
{
    static std::mutex mu;
    static std::map<int, lp_ctx *> ctxs;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    lp_ctx *ctx = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = ctxs.find(dev);
        if (it == ctxs.end()) {
            int rc = lp_ctx_create(&ctx, dev);
            if (rc != LP_OK) return rc;
            ctxs[dev] = ctx;
        } else {
            ctx = it->second;
        }
        lp_options o;
        lp_options_init(&o);
        o.flags = LP_FLAG_SYNC;
        return lp_batch_solve_ex(ctx, num_lps, A, b, c, sense, m, n, status, x, obj, &o);
    }
}

}  // extern "C"
