// ctx.h -- host-side pieces shared by the runtime's source files: the context
// (lp_ctx), grow-only device buffers, error reporting and kernel timers.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "lpbatch.h"

namespace lpb {

extern thread_local std::string g_last_error;

// Records the text of a failure for lp_last_error and returns `code`.
inline int fail(int code, const char *fmt, ...)
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
            return ::lpb::fail(LP_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Grow-only device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    int ensure(size_t need)
    {
        if (need <= bytes) return LP_OK;
        // Work queued earlier may still use the old buffer: let it finish first.
        if (p) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p);
        }
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
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as(size_t byte_off = 0) const { return reinterpret_cast<T *>(static_cast<char *>(p) + byte_off); }
};

struct KernelTime {
    const char *name;
    hipEvent_t start, stop;
};

// State of the warm-start network on one device.
struct MlpState {
    bool ready = false;        // parameters initialised or loaded
    int64_t step = 0;          // AdamW steps taken
    DevBuf params, params16;   // FP32 master [LP_MLP_NUM_PARAMS], BF16 copy
    DevBuf adam_m, adam_v, grads;
    DevBuf act;                // activations of the last batch
    DevBuf misc;               // loss scalar
};

// Grow-only pinned host buffer (hipHostMalloc).
struct PinnedBuf {
    void *p = nullptr;
    size_t bytes = 0;
    int ensure(size_t need)
    {
        if (need <= bytes) return LP_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        size_t want = std::max(need, size_t(4096));
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            return fail(LP_ERR_NOMEM, "hipHostMalloc of %zu bytes failed", want);
        }
        bytes = want;
        return LP_OK;
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// One of the rotating chunk buffers of lp_batch_solve_host: the chunk's device
// arrays, pinned staging for pageable caller memory, and the events that order
// upload -> solve -> download.
struct PipeSet {
    DevBuf dev;                 // A | b | c | sense | status | x | obj
    PinnedBuf in, out;          // staging of inputs / outputs
    hipEvent_t up = nullptr, solved = nullptr, down = nullptr;
    bool pending = false;       // a download not yet collected
    int64_t first = 0, count = 0;
};

struct HostPipe {
    bool ready = false;
    hipStream_t h2d = nullptr, comp = nullptr, d2h = nullptr;
    PipeSet set[3];
};

// Tuned launch of one size bin of the workgroup kernel.
struct TuneEntry {
    int nt;         // workgroup size
    int force_hbm;  // 1: tableaux in device-memory slots; 0: in LDS whenever they fit
};

inline int tune_key(int bin, bool fp32) { return bin * 2 + (fp32 ? 1 : 0); }

// The device metadata of the last batch of mixed LP sizes that was planned
// (shapes, offsets, id lists, in the context's `meta` buffer): a solve of the
// same shapes reuses it without an upload, so repeat solves queue their kernels
// without waiting on the host and can be captured in a HIP graph.  Uploads go
// through a pinned staging buffer; the event lets the next upload wait until
// the previous one has read it.
struct PlanCache {
    bool valid = false;
    uint64_t hash = 0;          // of num, m[], n[] and the planning flags
    const void *meta_p = nullptr;
    size_t meta_bytes = 0;
    PinnedBuf staging;
    hipEvent_t uploaded = nullptr;
};

}  // namespace lpb

struct lp_ctx {
    int device = 0;
    bool counters_dirty = false;  // a failed call may have left work counters non-zero
    int num_cu = 0;
    int max_lds = 0;
    int lds_per_cu = 0;  // LDS of one compute unit, shared by its resident workgroups
    lpb::DevBuf scratch, meta, counters;
    lpb::DevBuf scaled, scale_meta;  // lp_options.scaling: scaled copy, shapes
    std::vector<lpb::KernelTime> times;
    std::vector<hipEvent_t> event_pool;
    size_t events_used = 0;
    lpb::MlpState mlp;
    std::map<int, lpb::TuneEntry> tune;  // size bin x precision -> launch (autotuner)
    lpb::HostPipe pipe;                  // lp_batch_solve_host streams and buffers
    lpb::PlanCache plan;                 // uploaded metadata of the last mixed-size batch
    void *noalloc = nullptr;             // this device's copy of lp_batch_solve_noalloc's scratch
    int noalloc_err = 0;                 // hipError_t of its address lookup
};

namespace lpb {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

inline hipEvent_t take_event(lp_ctx *ctx)
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
        (void)hipEventRecord(kt.start, s);
    }
    void done()
    {
        if (!on) return;
        (void)hipEventRecord(kt.stop, s);
        ctx->times.push_back(kt);
        on = false;
    }
};

}  // namespace lpb
