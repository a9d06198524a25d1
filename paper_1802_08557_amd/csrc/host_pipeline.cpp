// host_pipeline.cpp -- lp_batch_solve_host: a batch held in host memory,
// streamed through the device in chunks.
//
// The paper cuts a batch larger than the device into chunks (its batching
// routine, Algorithm 1: capacity = device memory / memory per LP, Eq. (5)),
// copies each over, solves it and copies the results back, and hides the
// copies behind the kernels with CUDA streams.  Here: three chunk buffers in
// rotation and three streams -- uploads on one, solves on another once their
// upload has arrived, downloads on the third once their solve is done -- so
// chunk i+1's upload and chunk i-1's download overlap chunk i's solve.  The
// calling thread stages pageable caller memory through pinned buffers (in
// parallel slices) while the device works on the previous chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "ctx.h"
#include "lpbatch.h"

using lpb::fail;

namespace {

bool is_pinned(const void *p)
{
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();  // pageable memory may report an error; clear it
        return false;
    }
    return at.type == hipMemoryTypeHost;
}

// memcpy in up to eight slices on their own threads for large copies.
void parallel_copy(void *dst, const void *src, size_t bytes)
{
    constexpr size_t kSlice = size_t(8) << 20;
    if (bytes <= kSlice) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t parts = std::min<size_t>({size_t(8), size_t(hw), (bytes + kSlice - 1) / kSlice});
    const size_t step = (bytes + parts - 1) / parts;
    std::vector<std::thread> th;
    th.reserve(parts);
    size_t done = 0;  // bytes handed to threads; the calling thread copies the rest
    try {
        for (size_t t = 0; t < parts; ++t) {
            const size_t lo = t * step, hi = std::min(bytes, lo + step);
            if (lo >= hi) break;
            th.emplace_back([=] {
                std::memcpy(static_cast<char *>(dst) + lo, static_cast<const char *>(src) + lo, hi - lo);
            });
            done = hi;
        }
    } catch (...) {
        // No thread could be started: the slices not handed out are copied here.
    }
    if (done < bytes) std::memcpy(static_cast<char *>(dst) + done, static_cast<const char *>(src) + done, bytes - done);
    for (auto &t : th) t.join();
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Byte layout of one chunk's arrays (device buffer and staging alike).
struct ChunkLayout {
    size_t A, b, c, sense, status, x, obj;  // offsets
    size_t in_bytes, out_bytes, dev_bytes;
};

ChunkLayout layout(int64_t max_mn, int64_t max_m, int64_t max_n, int64_t max_lps)
{
    ChunkLayout L{};
    L.A = 0;
    L.b = align256(8 * size_t(max_mn));
    L.c = L.b + align256(8 * size_t(max_m));
    L.sense = L.c + align256(8 * size_t(max_n));
    L.in_bytes = L.sense + align256(size_t(max_m));
    L.status = 0;
    L.x = align256(4 * size_t(max_lps));
    L.obj = L.x + align256(8 * size_t(max_n));
    L.out_bytes = L.obj + align256(8 * size_t(max_lps));
    L.dev_bytes = L.in_bytes + L.out_bytes;
    return L;
}

int ensure_pipe(lp_ctx *ctx)
{
    lpb::HostPipe &H = ctx->pipe;
    if (H.ready) return LP_OK;
    // Default-priority streams that do not synchronise with the null stream.
    for (hipStream_t *st : {&H.h2d, &H.comp, &H.d2h})
        if (!*st) HIP_TRY(hipStreamCreateWithFlags(st, hipStreamNonBlocking));
    for (lpb::PipeSet &S : H.set)
        for (hipEvent_t *e : {&S.up, &S.solved, &S.down})
            if (!*e) HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
    H.ready = true;
    return LP_OK;
}

struct Caller {
    const double *A, *b, *c;
    const int8_t *sense;
    int32_t *status;
    double *x, *obj;
    bool pin_in[4], pin_out[3];
    const std::vector<int64_t> *ao, *ro, *co;
};

// Waits for set S's download and moves its results to the caller's arrays
// (a direct download into pinned caller memory needs no copy).
int collect(lpb::PipeSet &S, const ChunkLayout &L, const Caller &C)
{
    if (!S.pending) return LP_OK;
    HIP_TRY(hipEventSynchronize(S.down));
    S.pending = false;
    const int64_t f = S.first, e = S.first + S.count;
    const char *out = static_cast<const char *>(S.out.p);
    if (!C.pin_out[0]) std::memcpy(C.status + f, out + L.status, 4 * size_t(S.count));
    if (!C.pin_out[1])
        parallel_copy(C.x + (*C.co)[f], out + L.x, 8 * size_t((*C.co)[e] - (*C.co)[f]));
    if (!C.pin_out[2]) std::memcpy(C.obj + f, out + L.obj, 8 * size_t(S.count));
    return LP_OK;
}

}  // namespace

extern "C" int lp_batch_solve_host(lp_ctx *ctx, int64_t num_lps, const double *A, const double *b,
                                   const double *c, const int8_t *sense, const int32_t *m,
                                   const int32_t *n, int32_t *status, double *x, double *obj,
                                   const lp_options *opts_in, int64_t chunk_lps)
{
    if (!ctx) return fail(LP_ERR_ARG, "lp_batch_solve_host: ctx is NULL");
    if (num_lps < 0) return fail(LP_ERR_ARG, "num_lps is negative (%lld)", (long long)num_lps);
    if (chunk_lps < 0) return fail(LP_ERR_ARG, "chunk_lps is negative (%lld)", (long long)chunk_lps);
    lp_options opts;
    lp_options_init(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.stats || opts.shared || opts.row_subset)
        return fail(LP_ERR_ARG, "lp_batch_solve_host: stats, shared and row_subset are not supported");
    if (num_lps == 0) return LP_OK;
    if (!A || !b || !c || !sense || !m || !n || !status || !x || !obj)
        return fail(LP_ERR_ARG, "a batch pointer is NULL");
    if (num_lps > INT32_MAX) return fail(LP_ERR_ARG, "num_lps exceeds 2^31-1");

    // Offsets of every LP in the caller's concatenated arrays.
    std::vector<int64_t> ao(num_lps + 1), ro(num_lps + 1), co(num_lps + 1);
    for (int64_t k = 0; k < num_lps; ++k) {
        if (m[k] < 1 || n[k] < 1 || m[k] > 1000000 || n[k] > 1000000)
            return fail(LP_ERR_ARG, "LP %lld has m=%d n=%d", (long long)k, m[k], n[k]);
        ao[k + 1] = ao[k] + int64_t(m[k]) * n[k];
        ro[k + 1] = ro[k] + m[k];
        co[k + 1] = co[k] + n[k];
    }

    lpb::DeviceGuard g(ctx->device);
    // Chunk size: Eq. (5)-style capacity (device bytes per LP against a quarter
    // of the free memory, over three chunk buffers), and at least eight chunks
    // for the overlap unless that makes chunks smaller than 4096 LPs.
    const double per_lp = double(8 * ao[num_lps] + 9 * ro[num_lps] + 16 * co[num_lps] + 12 * num_lps) /
                          double(num_lps);
    if (chunk_lps == 0) {
        size_t free_b = 0, total_b = 0;
        HIP_TRY(hipMemGetInfo(&free_b, &total_b));
        const int64_t cap = std::max<int64_t>(1, int64_t(double(free_b) / 4.0 / 3.0 / per_lp));
        chunk_lps = std::min(cap, std::max<int64_t>(4096, (num_lps + 7) / 8));
    }
    chunk_lps = std::min(chunk_lps, num_lps);
    const int64_t nchunks = (num_lps + chunk_lps - 1) / chunk_lps;
    int64_t max_mn = 0, max_m = 0, max_n = 0;
    for (int64_t i = 0; i < nchunks; ++i) {
        const int64_t f = i * chunk_lps, e = std::min(num_lps, f + chunk_lps);
        max_mn = std::max(max_mn, ao[e] - ao[f]);
        max_m = std::max(max_m, ro[e] - ro[f]);
        max_n = std::max(max_n, co[e] - co[f]);
    }
    const ChunkLayout L = layout(max_mn, max_m, max_n, chunk_lps);

    Caller C{A, b, c, sense, status, x, obj, {}, {}, &ao, &ro, &co};
    C.pin_in[0] = is_pinned(A);
    C.pin_in[1] = is_pinned(b);
    C.pin_in[2] = is_pinned(c);
    C.pin_in[3] = is_pinned(sense);
    C.pin_out[0] = is_pinned(status);
    C.pin_out[1] = is_pinned(x);
    C.pin_out[2] = is_pinned(obj);
    const bool stage_in = !(C.pin_in[0] && C.pin_in[1] && C.pin_in[2] && C.pin_in[3]);
    const bool stage_out = !(C.pin_out[0] && C.pin_out[1] && C.pin_out[2]);

    int rc = ensure_pipe(ctx);
    if (rc != LP_OK) return rc;
    lpb::HostPipe &H = ctx->pipe;
    const int nsets = int(std::min<int64_t>(3, nchunks));
    for (int j = 0; j < nsets; ++j) {
        lpb::PipeSet &S = H.set[j];
        S.pending = false;
        if ((rc = S.dev.ensure(L.dev_bytes)) != LP_OK) return rc;
        if (stage_in && (rc = S.in.ensure(L.in_bytes)) != LP_OK) return rc;
        if (stage_out && (rc = S.out.ensure(L.out_bytes)) != LP_OK) return rc;
    }
    opts.stream = H.comp;
    opts.flags &= ~LP_FLAG_SYNC;

    auto drain = [&](int64_t upto) {
        // Collect every pending set (in chunk order), keeping the first error.
        int r = LP_OK;
        for (int64_t i = std::max<int64_t>(0, upto - 3); i < upto; ++i) {
            const int q = collect(H.set[i % 3], L, C);
            if (r == LP_OK) r = q;
        }
        return r;
    };
    // On a failure: let the queued copies and solves finish (they use the
    // context's buffers), forget the pending downloads, return the error.
    auto bail = [&](int r) {
        for (hipStream_t st : {H.h2d, H.comp, H.d2h}) (void)hipStreamSynchronize(st);
        for (lpb::PipeSet &S : H.set) S.pending = false;
        return r;
    };
#define PIPE_TRY(expr)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return bail(fail(LP_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)));     \
    } while (0)

    for (int64_t i = 0; i < nchunks; ++i) {
        lpb::PipeSet &S = H.set[i % 3];
        if ((rc = collect(S, L, C)) != LP_OK) return bail(rc);
        const int64_t f = i * chunk_lps, e = std::min(num_lps, f + chunk_lps), cnt = e - f;
        char *dev = S.dev.as<char>();
        char *dout = dev + L.in_bytes;
        const size_t bA = 8 * size_t(ao[e] - ao[f]), bR = size_t(ro[e] - ro[f]), bC = 8 * size_t(co[e] - co[f]);
        const void *src[4] = {A + ao[f], b + ro[f], c + co[f], sense + ro[f]};
        const size_t off[4] = {L.A, L.b, L.c, L.sense}, len[4] = {bA, 8 * bR, bC, bR};
        for (int t = 0; t < 4; ++t) {
            const void *up = src[t];
            if (!C.pin_in[t]) {
                char *stg = static_cast<char *>(S.in.p) + off[t];
                parallel_copy(stg, src[t], len[t]);
                up = stg;
            }
            if (len[t]) PIPE_TRY(hipMemcpyAsync(dev + off[t], up, len[t], hipMemcpyHostToDevice, H.h2d));
        }
        PIPE_TRY(hipEventRecord(S.up, H.h2d));
        PIPE_TRY(hipStreamWaitEvent(H.comp, S.up, 0));
        rc = lp_batch_solve_ex(ctx, cnt, reinterpret_cast<const double *>(dev + L.A),
                               reinterpret_cast<const double *>(dev + L.b),
                               reinterpret_cast<const double *>(dev + L.c),
                               reinterpret_cast<const int8_t *>(dev + L.sense), m + f, n + f,
                               reinterpret_cast<int32_t *>(dout + L.status), reinterpret_cast<double *>(dout + L.x),
                               reinterpret_cast<double *>(dout + L.obj), &opts);
        if (rc != LP_OK) return bail(rc);
        PIPE_TRY(hipEventRecord(S.solved, H.comp));
        PIPE_TRY(hipStreamWaitEvent(H.d2h, S.solved, 0));
        void *dst[3] = {C.pin_out[0] ? static_cast<void *>(status + f) : static_cast<char *>(S.out.p) + L.status,
                        C.pin_out[1] ? static_cast<void *>(x + co[f]) : static_cast<char *>(S.out.p) + L.x,
                        C.pin_out[2] ? static_cast<void *>(obj + f) : static_cast<char *>(S.out.p) + L.obj};
        const size_t doff[3] = {L.status, L.x, L.obj}, dlen[3] = {4 * size_t(cnt), bC, 8 * size_t(cnt)};
        for (int t = 0; t < 3; ++t) PIPE_TRY(hipMemcpyAsync(dst[t], dout + doff[t], dlen[t], hipMemcpyDeviceToHost, H.d2h));
        PIPE_TRY(hipEventRecord(S.down, H.d2h));
        S.pending = true;
        S.first = f;
        S.count = cnt;
    }
    rc = drain(nchunks);
#undef PIPE_TRY
    return rc == LP_OK ? LP_OK : bail(rc);
}
