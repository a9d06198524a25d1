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

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(LP_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

// Grow-only device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    int ensure(size_t need)
    {
        if (need <= bytes) return LP_OK;
        if (p) hipFree(p);
        p = nullptr;
        bytes = 0;
        size_t want = std::max(need, size_t(4096));
        if (hipMalloc(&p, want) != hipSuccess) {
            p = nullptr;
            return fail(LP_ERR_NOMEM, "hipMalloc of %zu bytes failed", want);
        }
        bytes = want;
        return LP_OK;
    }
    void release()
    {
        if (p) hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

struct KernelTime {
    const char *name;
    hipEvent_t start, stop;
};

}  // namespace

struct lp_ctx {
    int device = 0;
    int num_cu = 0;
    int max_lds = 0;
    DevBuf scratch, meta, counters;
    std::vector<KernelTime> times;
    std::vector<hipEvent_t> event_pool;
    size_t events_used = 0;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        hipGetDevice(&prev);
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) hipSetDevice(prev);
    }
};

hipEvent_t take_event(lp_ctx *ctx)
{
    if (ctx->events_used == ctx->event_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->event_pool.push_back(e);
    }
    return ctx->event_pool[ctx->events_used++];
}

// Records kernel timing events around a launch when asked to.
struct Timer {
    lp_ctx *ctx;
    bool on;
    hipStream_t s;
    KernelTime kt{};
    Timer(lp_ctx *c, bool enabled, hipStream_t st, const char *name) : ctx(c), on(enabled), s(st)
    {
        if (!on) return;
        kt.name = name;
        kt.start = take_event(ctx);
        kt.stop = take_event(ctx);
        if (!kt.start || !kt.stop) { on = false; return; }
        hipEventRecord(kt.start, s);
    }
    void done()
    {
        if (!on) return;
        hipEventRecord(kt.stop, s);
        ctx->times.push_back(kt);
        on = false;
    }
};

lpb::SolveParams fill_params(const lp_options &o, bool fp32)
{
    lpb::SolveParams p;
    p.tol_piv = o.tol_piv > 0 ? o.tol_piv : (fp32 ? 1e-6 : 1e-9);
    p.tol_opt = o.tol_opt > 0 ? o.tol_opt : (fp32 ? 1e-6 : 1e-9);
    p.tol_feas = o.tol_feas > 0 ? o.tol_feas : (fp32 ? 1e-6 : 1e-9);
    p.k_deg = o.k_deg == 0 ? 50 : o.k_deg;
    p.max_iters = o.max_iters;
    return p;
}

}  // namespace

extern "C" {

const char *lp_last_error(void) { return g_last_error.c_str(); }

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
    if (e1 != hipSuccess || e2 != hipSuccess) {
        delete ctx;
        return fail(LP_ERR_HIP, "lp_ctx_create: device attribute query failed");
    }
    if (lpb::simplex_configure(ctx->max_lds) != hipSuccess ||
        lpb::simplex_wave_configure(ctx->max_lds) != hipSuccess) {
        delete ctx;
        return fail(LP_ERR_HIP, "lp_ctx_create: could not configure kernel LDS limits");
    }
    int rc = ctx->counters.ensure(4096);
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
    hipDeviceSynchronize();
    ctx->scratch.release();
    ctx->meta.release();
    ctx->counters.release();
    for (hipEvent_t e : ctx->event_pool) hipEventDestroy(e);
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
    if (num_lps == 0) return LP_OK;
    if (!A || !b || !c || !sense || !m || !n || !status || !x || !obj)
        return fail(LP_ERR_ARG, "a batch pointer is NULL");
    if (num_lps > INT32_MAX) return fail(LP_ERR_ARG, "num_lps exceeds 2^31-1");

    // Shapes (host arrays), offsets and the uniform-shape shortcut.
    int32_t m0 = m[0], n0 = n[0], m_max = 0, n_max = 0;
    bool uniform = true;
    int64_t sa = 0, sr = 0, sc = 0;
    for (int64_t k = 0; k < num_lps; ++k) {
        const int32_t mk = m[k], nk = n[k];
        if (mk < 1 || nk < 1)
            return fail(LP_ERR_ARG, "LP %lld has m=%d n=%d (both must be >= 1)", (long long)k, mk, nk);
        if (mk > 1000000 || nk > 1000000)
            return fail(LP_ERR_ARG, "LP %lld is too large (m=%d n=%d)", (long long)k, mk, nk);
        uniform = uniform && mk == m0 && nk == n0;
        m_max = std::max(m_max, mk);
        n_max = std::max(n_max, nk);
        sa += int64_t(mk) * nk;
        sr += mk;
        sc += nk;
        if (sa < 0 || sa > (int64_t(1) << 60)) return fail(LP_ERR_ARG, "batch size overflows");
    }
    const bool fp32 = opts.precision == LP_PREC_FP32_CERT64;
    if (fp32) return fail(LP_ERR_ARG, "LP_PREC_FP32_CERT64 is not available in this build");
    hipStream_t stream = reinterpret_cast<hipStream_t>(opts.stream);
    DeviceGuard g(ctx->device);
    const int64_t ts = fp32 ? 4 : 8;

    // Kernel choice per LP: one wavefront for LPs of at most 63 columns and 128
    // rows whose tableau fits LDS, a workgroup otherwise (or when the caller
    // fixes the workgroup size or asks for HBM placement).
    const bool auto_kernel = opts.block_threads == 0 && opts.placement != LP_PLACE_HBM;
    auto wave_fit = [&](int64_t mk, int64_t nk) {
        return nk <= 63 && mk <= 128 &&
               lpb::wave_lds_aux_bytes(mk > 64 ? 2 : 1, fp32) + mk * lpb::tableau_ld(int(nk) + 1) * ts <=
                   ctx->max_lds;
    };
    std::vector<int32_t> wave_ids, block_ids;
    int64_t n_wave = 0;
    int wm_max = 0, wn_max = 0;
    for (int64_t k = 0; k < num_lps; ++k) {
        const bool w = auto_kernel && wave_fit(m[k], n[k]);
        if (w) {
            ++n_wave;
            wm_max = std::max(wm_max, m[k]);
            wn_max = std::max(wn_max, n[k]);
        }
        if (!uniform) (w ? wave_ids : block_ids).push_back(int32_t(k));
    }
    const int64_t n_block = num_lps - n_wave;

    lpb::SolveArgs a;
    std::memset(&a, 0, sizeof a);
    a.A = A; a.b = b; a.c = c; a.sense = sense;
    a.status = status; a.x = x; a.obj = obj;
    a.stats = opts.stats;
    a.prm = fill_params(opts, fp32);

    // Device metadata: [m][n][aoff][roff][coff] (non-uniform only), then the
    // wavefront id list and the deferred/workgroup id list (capacity num_lps).
    const size_t sz_shape = uniform ? 0 : size_t(num_lps) * (2 * sizeof(int32_t) + 3 * sizeof(int64_t));
    const size_t sz_ids = size_t(num_lps) * sizeof(int32_t);
    {
        int rc = ctx->meta.ensure(sz_shape + 2 * sz_ids);
        if (rc != LP_OK) return rc;
    }
    char *meta = static_cast<char *>(ctx->meta.p);
    int32_t *d_wave_ids = reinterpret_cast<int32_t *>(meta + sz_shape);
    int32_t *d_defer_ids = d_wave_ids + num_lps;
    if (uniform) {
        a.um = m0;
        a.un = n0;
    } else {
        std::vector<char> host(sz_shape + sz_ids + size_t(n_block) * sizeof(int32_t));
        int32_t *hm = reinterpret_cast<int32_t *>(host.data());
        int32_t *hn = hm + num_lps;
        int64_t *ha = reinterpret_cast<int64_t *>(hn + num_lps);
        int64_t *hr = ha + num_lps, *hc = hr + num_lps;
        int64_t oa = 0, orr = 0, oc = 0;
        for (int64_t k = 0; k < num_lps; ++k) {
            hm[k] = m[k]; hn[k] = n[k];
            ha[k] = oa; hr[k] = orr; hc[k] = oc;
            oa += int64_t(m[k]) * n[k]; orr += m[k]; oc += n[k];
        }
        int32_t *hw = reinterpret_cast<int32_t *>(host.data() + sz_shape);
        std::copy(wave_ids.begin(), wave_ids.end(), hw);
        int32_t *hb = hw + num_lps;
        std::copy(block_ids.begin(), block_ids.end(), hb);
        HIP_TRY(hipMemcpyAsync(meta, host.data(), host.size(), hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));  // the host staging buffer goes away
        a.m = reinterpret_cast<int32_t *>(meta);
        a.n = a.m + num_lps;
        a.aoff = reinterpret_cast<int64_t *>(const_cast<int32_t *>(a.n + num_lps));
        a.roff = a.aoff + num_lps;
        a.coff = a.roff + num_lps;
    }
    int32_t *cnt = static_cast<int32_t *>(ctx->counters.p);  // [0] wave queue, [1] block queue, [2] deferred
    const bool timing = (opts.flags & LP_FLAG_TIME_KERNELS) != 0;

    if (n_wave > 0) {
        const int rb = wm_max > 64 ? 2 : 1;
        lpb::SolveArgs w = a;
        w.num = n_wave;
        w.ids = uniform ? nullptr : d_wave_ids;
        w.queue = cnt;
        w.defer_ids = d_defer_ids;
        w.defer_count = cnt + 2;
        const int64_t lds = lpb::wave_lds_aux_bytes(rb, fp32) +
                            int64_t(wm_max) * lpb::tableau_ld(wn_max + 1) * ts;
        w.lds_bytes = int32_t(lds);
        const int per_cu = lpb::simplex_wave_blocks_per_cu(fp32, rb, int(lds));
        if (per_cu < 1) return fail(LP_ERR_HIP, "occupancy query failed for the wavefront kernel");
        const int64_t grid = std::min<int64_t>(n_wave, int64_t(per_cu) * ctx->num_cu);
        HIP_TRY(lpb::launch_zero_i32(cnt, 1, stream));
        HIP_TRY(lpb::launch_set_i32(cnt + 2, int32_t(n_block), stream));
        Timer t(ctx, timing, stream, fp32 ? "simplex_wave_fp32" : "simplex_wave_fp64");
        HIP_TRY(lpb::launch_simplex_wave(fp32, rb, w, int(grid), stream));
        t.done();
    }

    // Workgroup kernel: every LP not given to a wavefront, plus the deferred ones.
    const int ncol_worst = n_max + m_max;
    lpb::LdsLayout L = lpb::lds_layout(m_max, ncol_worst, ts, lpb::simplex_ctrl_bytes(fp32));
    // Tableau budget for the common case of no surplus columns (every row <= after
    // normalisation); LPs with more columns than budgeted move to HBM by themselves.
    const int64_t tab_common = int64_t(m_max + 1) * lpb::tableau_ld(n_max + 1) * ts;
    const int64_t tab_worst = int64_t(m_max + 1) * lpb::tableau_ld(ncol_worst + 1) * ts;
    const int64_t cells = int64_t(m_max + 1) * (n_max + 1);
    int nt = opts.block_threads;
    if (!nt) nt = cells <= 64 * 64 ? 64 : (cells <= 256 * 256 ? 256 : 512);
    int64_t lds = L.tab;
    const bool want_lds = opts.placement != LP_PLACE_HBM && L.tab + tab_common <= ctx->max_lds;
    if (want_lds) lds = L.tab + tab_common;
    if (lds > ctx->max_lds)
        return fail(LP_ERR_ARG, "LP of %d rows x %d columns needs %lld bytes of LDS for its index "
                    "arrays (device limit %d)", m_max, ncol_worst, (long long)lds, ctx->max_lds);
    a.lds_bytes = int32_t(lds);
    a.force_hbm = opts.placement == LP_PLACE_HBM;
    const int per_cu = lpb::simplex_blocks_per_cu(fp32, nt, int(lds));
    if (per_cu < 1) return fail(LP_ERR_HIP, "occupancy query failed for %d threads, %lld B LDS", nt, (long long)lds);
    const int64_t grid = std::min<int64_t>(num_lps, int64_t(per_cu) * ctx->num_cu);
    const bool need_hbm = !want_lds || tab_worst > tab_common;
    if (need_hbm) {
        a.slot_bytes = lpb::align16(tab_worst);
        int rc = ctx->scratch.ensure(size_t(a.slot_bytes) * size_t(grid));
        if (rc != LP_OK) return rc;
        a.scratch = static_cast<char *>(ctx->scratch.p);
    }
    a.queue = cnt + 1;
    if (n_wave > 0) {
        a.num = num_lps;  // upper bound; the deferred count is read on the device
        a.ids = d_defer_ids;
        a.num_dev = cnt + 2;
    } else {
        a.num = num_lps;
        a.ids = nullptr;
    }
    HIP_TRY(lpb::launch_zero_i32(cnt + 1, 1, stream));
    {
        Timer t(ctx, timing, stream, fp32 ? "simplex_block_fp32" : "simplex_block_fp64");
        HIP_TRY(lpb::launch_simplex(fp32, nt, a, int(grid), stream));
        t.done();
    }
    if (opts.flags & LP_FLAG_SYNC) HIP_TRY(hipStreamSynchronize(stream));
    return LP_OK;
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
