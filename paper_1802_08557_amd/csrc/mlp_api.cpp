// mlp_api.cpp -- host side of the warm-start network (lp_mlp_* in lpbatch.h).
//
// The network (20 -> 256 -> 256 -> 120, ReLU) keeps FP32 master parameters,
// a BF16 copy that feeds the matrix cores, and the AdamW moments in the
// context.  Each entry point queues its kernels on the caller's stream; the
// parameter buffers are reused by every call, so calls that use the network
// must be ordered on one stream (or synchronised) by the caller.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lpbatch.h"
#include "internal.h"
#include "ctx.h"

namespace {

using lpb::DevBuf;
using lpb::DeviceGuard;
using lpb::fail;

constexpr int IN = LP_MLP_IN, H = LP_MLP_HIDDEN, OUT = LP_MLP_OUT;
constexpr int64_t NP = LP_MLP_NUM_PARAMS;
// Offsets of the parameter blocks in the flat vector.
constexpr int64_t OW1 = 0, OB1 = OW1 + int64_t(H) * IN, OW2 = OB1 + H, OB2 = OW2 + int64_t(H) * H,
                  OW3 = OB2 + H, OB3 = OW3 + int64_t(OUT) * H;
static_assert(OB3 + OUT == NP, "parameter layout");

// Activation buffers of a batch of B rows (byte offsets into MlpState::act).
struct Act {
    size_t x16, z1, h1, z2, h2, s, ds, ds16, dz2, dz216, dz1, dz116, rowloss, total;
};

Act act_layout(int64_t B, bool train)
{
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    Act a{};
    size_t o = 0;
    a.x16 = o; o += al(size_t(B) * IN * 2);
    a.h1 = o; o += al(size_t(B) * H * 2);
    a.h2 = o; o += al(size_t(B) * H * 2);
    a.s = o; o += al(size_t(B) * OUT * 4);
    if (train) {
        a.z1 = o; o += al(size_t(B) * H * 4);
        a.z2 = o; o += al(size_t(B) * H * 4);
        a.ds = o; o += al(size_t(B) * OUT * 4);
        a.ds16 = o; o += al(size_t(B) * OUT * 2);
        a.dz2 = o; o += al(size_t(B) * H * 4);
        a.dz216 = o; o += al(size_t(B) * H * 2);
        a.dz1 = o; o += al(size_t(B) * H * 4);
        a.dz116 = o; o += al(size_t(B) * H * 2);
        a.rowloss = o; o += al(size_t(B) * 4);
    }
    a.total = o;
    return a;
}

int check_ready(lp_ctx *ctx)
{
    if (!ctx) return fail(LP_ERR_ARG, "ctx is NULL");
    if (!ctx->mlp.ready) return fail(LP_ERR_ARG, "the network has no parameters (call lp_mlp_init or lp_mlp_load)");
    return LP_OK;
}

int alloc_params(lp_ctx *ctx)
{
    lpb::MlpState &M = ctx->mlp;
    for (DevBuf *d : {&M.params, &M.adam_m, &M.adam_v, &M.grads}) {
        int rc = d->ensure(size_t(NP) * 4);
        if (rc != LP_OK) return rc;
    }
    int rc = M.params16.ensure(size_t(NP) * 2);
    if (rc == LP_OK) rc = M.misc.ensure(256);
    return rc;
}

// Fresh AdamW state and BF16 copy after new master parameters.
int reset_state(lp_ctx *ctx, hipStream_t s)
{
    lpb::MlpState &M = ctx->mlp;
    HIP_TRY(hipMemsetAsync(M.adam_m.p, 0, size_t(NP) * 4, s));
    HIP_TRY(hipMemsetAsync(M.adam_v.p, 0, size_t(NP) * 4, s));
    HIP_TRY(lpb::launch_cast_params(M.params.as<float>(), M.params16.as<uint16_t>(), NP, s));
    M.step = 0;
    M.ready = true;
    return LP_OK;
}

lpb::MlpGemm gemm(int M, int N, int K, const uint16_t *a, int64_t sai, int64_t sak, const uint16_t *b,
                  int64_t sbk, int64_t sbj)
{
    lpb::MlpGemm g;
    std::memset(&g, 0, sizeof g);
    g.M = M; g.N = N; g.K = K;
    g.a = a; g.sai = sai; g.sak = sak;
    g.b = b; g.sbk = sbk; g.sbj = sbj;
    g.ldc = N;
    return g;
}

// Forward pass of B rows; training keeps Z1, Z2 for the backward pass.
int forward(lp_ctx *ctx, int64_t B, const float *dirs, const Act &L, bool train, hipStream_t s)
{
    lpb::MlpState &M = ctx->mlp;
    char *act = M.act.as<char>();
    const uint16_t *w16 = M.params16.as<uint16_t>();
    const float *w = M.params.as<float>();
    uint16_t *x16 = reinterpret_cast<uint16_t *>(act + L.x16);
    uint16_t *h1 = reinterpret_cast<uint16_t *>(act + L.h1);
    uint16_t *h2 = reinterpret_cast<uint16_t *>(act + L.h2);
    HIP_TRY(lpb::launch_to_bf16(dirs, x16, B * IN, s));
    const int Bi = int(B);
    lpb::MlpGemm g = gemm(Bi, H, IN, x16, IN, 1, w16 + OW1, 1, IN);
    g.bias = w + OB1;
    g.c32 = train ? reinterpret_cast<float *>(act + L.z1) : nullptr;
    g.c16 = h1;
    g.relu = 1;
    HIP_TRY(lpb::launch_mlp_gemm(g, s));
    g = gemm(Bi, H, H, h1, H, 1, w16 + OW2, 1, H);
    g.bias = w + OB2;
    g.c32 = train ? reinterpret_cast<float *>(act + L.z2) : nullptr;
    g.c16 = h2;
    g.relu = 1;
    HIP_TRY(lpb::launch_mlp_gemm(g, s));
    g = gemm(Bi, OUT, H, h2, H, 1, w16 + OW3, 1, H);
    g.bias = w + OB3;
    g.c32 = reinterpret_cast<float *>(act + L.s);
    HIP_TRY(lpb::launch_mlp_gemm(g, s));
    return LP_OK;
}

// Loss and gradients of B labelled rows into M.grads and M.misc[0].
int loss_grads(lp_ctx *ctx, int64_t B, const float *dirs, const uint8_t *tight, hipStream_t s)
{
    lpb::MlpState &M = ctx->mlp;
    const Act L = act_layout(B, true);
    int rc = M.act.ensure(L.total);
    if (rc != LP_OK) return rc;
    rc = forward(ctx, B, dirs, L, true, s);
    if (rc != LP_OK) return rc;
    char *act = M.act.as<char>();
    auto f32 = [&](size_t o) { return reinterpret_cast<float *>(act + o); };
    auto b16 = [&](size_t o) { return reinterpret_cast<uint16_t *>(act + o); };
    const uint16_t *w16 = M.params16.as<uint16_t>();
    float *gr = M.grads.as<float>();
    const int Bi = int(B);
    HIP_TRY(lpb::launch_bce(f32(L.s), tight, B, OUT, f32(L.ds), b16(L.ds16), f32(L.rowloss), M.misc.as<float>(), s));
    // dW3 = q(dS)^T H2, db3 = column sums of dS.
    lpb::MlpGemm g = gemm(OUT, H, Bi, b16(L.ds16), 1, OUT, b16(L.h2), H, 1);
    g.c32 = gr + OW3;
    HIP_TRY(lpb::launch_mlp_gemm(g, s));
    HIP_TRY(lpb::launch_colsum(f32(L.ds), B, OUT, gr + OB3, s));
    // dZ2 = (q(dS) q(W3)) * [Z2 > 0].
    g = gemm(Bi, H, OUT, b16(L.ds16), OUT, 1, w16 + OW3, H, 1);
    g.mask = f32(L.z2);
    g.c32 = f32(L.dz2);
    g.c16 = b16(L.dz216);
    HIP_TRY(lpb::launch_mlp_gemm(g, s));
    // dW2 = q(dZ2)^T H1, db2.
    g = gemm(H, H, Bi, b16(L.dz216), 1, H, b16(L.h1), H, 1);
    g.c32 = gr + OW2;
    HIP_TRY(lpb::launch_mlp_gemm(g, s));
    HIP_TRY(lpb::launch_colsum(f32(L.dz2), B, H, gr + OB2, s));
    // dZ1 = (q(dZ2) q(W2)) * [Z1 > 0].
    g = gemm(Bi, H, H, b16(L.dz216), H, 1, w16 + OW2, H, 1);
    g.mask = f32(L.z1);
    g.c32 = f32(L.dz1);
    g.c16 = b16(L.dz116);
    HIP_TRY(lpb::launch_mlp_gemm(g, s));
    // dW1 = q(dZ1)^T X, db1.
    g = gemm(H, IN, Bi, b16(L.dz116), 1, H, b16(L.x16), IN, 1);
    g.c32 = gr + OW1;
    HIP_TRY(lpb::launch_mlp_gemm(g, s));
    HIP_TRY(lpb::launch_colsum(f32(L.dz1), B, H, gr + OB1, s));
    return LP_OK;
}

int check_batch(int64_t B, const void *dirs)
{
    if (B < 1) return fail(LP_ERR_ARG, "batch size %lld must be >= 1", (long long)B);
    if (B > (int64_t(1) << 26)) return fail(LP_ERR_ARG, "batch size %lld too large", (long long)B);
    if (!dirs) return fail(LP_ERR_ARG, "dirs is NULL");
    return LP_OK;
}

// splitmix64 (Steele, Lea & Flood 2014): a counter-based 64-bit generator.
uint64_t splitmix64(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int lp_mlp_init(lp_ctx *ctx, uint64_t seed)
{
    if (!ctx) return fail(LP_ERR_ARG, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    int rc = alloc_params(ctx);
    if (rc != LP_OK) return rc;
    // He-uniform weights U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)); zero biases.
    std::vector<float> h(NP, 0.f);
    uint64_t st = seed;
    auto fill = [&](int64_t off, int64_t count, int fan_in) {
        const double r = std::sqrt(6.0 / fan_in);
        for (int64_t i = 0; i < count; ++i) {
            const double u = double(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
            h[off + i] = float((2.0 * u - 1.0) * r);
        }
    };
    fill(OW1, int64_t(H) * IN, IN);
    fill(OW2, int64_t(H) * H, H);
    fill(OW3, int64_t(OUT) * H, H);
    HIP_TRY(hipMemcpy(ctx->mlp.params.p, h.data(), size_t(NP) * 4, hipMemcpyHostToDevice));
    rc = reset_state(ctx, nullptr);
    if (rc != LP_OK) return rc;
    HIP_TRY(hipStreamSynchronize(nullptr));
    return LP_OK;
}

int lp_mlp_set_params(lp_ctx *ctx, const float *params, void *stream)
{
    if (!ctx) return fail(LP_ERR_ARG, "ctx is NULL");
    if (!params) return fail(LP_ERR_ARG, "params is NULL");
    DeviceGuard dg(ctx->device);
    int rc = alloc_params(ctx);
    if (rc != LP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(ctx->mlp.params.p, params, size_t(NP) * 4, hipMemcpyDeviceToDevice, s));
    return reset_state(ctx, s);
}

int lp_mlp_get_params(lp_ctx *ctx, float *params, void *stream)
{
    int rc = check_ready(ctx);
    if (rc != LP_OK) return rc;
    if (!params) return fail(LP_ERR_ARG, "params is NULL");
    DeviceGuard dg(ctx->device);
    HIP_TRY(hipMemcpyAsync(params, ctx->mlp.params.p, size_t(NP) * 4, hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)));
    return LP_OK;
}

int lp_mlp_infer(lp_ctx *ctx, int64_t B, const float *dirs, float *scores, int32_t *top_k, int32_t k,
                 void *stream)
{
    int rc = check_ready(ctx);
    if (rc != LP_OK) return rc;
    rc = check_batch(B, dirs);
    if (rc != LP_OK) return rc;
    if (top_k && (k < 1 || k > OUT)) return fail(LP_ERR_ARG, "k = %d must lie in 1..%d", k, OUT);
    if (!top_k && !scores) return fail(LP_ERR_ARG, "neither scores nor top_k requested");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // One fused kernel: no activations leave the chip.
    HIP_TRY(lpb::launch_mlp_infer(dirs, B, ctx->mlp.params16.as<uint16_t>(), ctx->mlp.params.as<float>(), scores,
                                  top_k, top_k ? k : 0, s));
    return LP_OK;
}

int lp_mlp_grads(lp_ctx *ctx, int64_t B, const float *dirs, const uint8_t *tight, float *grad_out,
                 float *loss_out, void *stream)
{
    int rc = check_ready(ctx);
    if (rc != LP_OK) return rc;
    rc = check_batch(B, dirs);
    if (rc != LP_OK) return rc;
    if (!tight) return fail(LP_ERR_ARG, "tight is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = loss_grads(ctx, B, dirs, tight, s);
    if (rc != LP_OK) return rc;
    if (grad_out) HIP_TRY(hipMemcpyAsync(grad_out, ctx->mlp.grads.p, size_t(NP) * 4, hipMemcpyDeviceToDevice, s));
    if (loss_out) HIP_TRY(hipMemcpyAsync(loss_out, ctx->mlp.misc.p, 4, hipMemcpyDeviceToDevice, s));
    return LP_OK;
}

int lp_mlp_train_step(lp_ctx *ctx, int64_t B, const float *dirs, const uint8_t *tight, float lr,
                      float weight_decay, float *loss_out, void *stream)
{
    int rc = check_ready(ctx);
    if (rc != LP_OK) return rc;
    rc = check_batch(B, dirs);
    if (rc != LP_OK) return rc;
    if (!tight) return fail(LP_ERR_ARG, "tight is NULL");
    if (!(lr >= 0.f) || !(weight_decay >= 0.f)) return fail(LP_ERR_ARG, "lr and weight_decay must be >= 0");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = loss_grads(ctx, B, dirs, tight, s);
    if (rc != LP_OK) return rc;
    lpb::MlpState &M = ctx->mlp;
    M.step += 1;
    lpb::MlpAdam h;
    h.lr = lr;
    h.wd = weight_decay;
    h.beta1 = 0.9f;
    h.beta2 = 0.999f;
    h.eps = 1e-8f;
    h.bc1 = float(1.0 - std::pow(0.9, double(M.step)));
    h.bc2 = float(1.0 - std::pow(0.999, double(M.step)));
    const int64_t decay[6] = {OW1, OB1, OW2, OB2, OW3, OB3};
    HIP_TRY(lpb::launch_adamw(M.params.as<float>(), M.grads.as<float>(), M.adam_m.as<float>(),
                              M.adam_v.as<float>(), M.params16.as<uint16_t>(), NP, h, decay, s));
    if (loss_out) HIP_TRY(hipMemcpyAsync(loss_out, M.misc.p, 4, hipMemcpyDeviceToDevice, s));
    return LP_OK;
}

int lp_mlp_save(lp_ctx *ctx, const char *path)
{
    int rc = check_ready(ctx);
    if (rc != LP_OK) return rc;
    if (!path) return fail(LP_ERR_ARG, "path is NULL");
    DeviceGuard dg(ctx->device);
    std::vector<float> buf(size_t(NP) * 3);
    lpb::MlpState &M = ctx->mlp;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(buf.data(), M.params.p, size_t(NP) * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(buf.data() + NP, M.adam_m.p, size_t(NP) * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(buf.data() + 2 * NP, M.adam_v.p, size_t(NP) * 4, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(LP_ERR_ARG, "cannot open %s for writing", path);
    const char magic[8] = {'L', 'P', 'M', 'L', 'P', '0', '0', '1'};
    const int64_t hdr[2] = {NP, M.step};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 8, 2, f) == 2 &&
              std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(LP_ERR_ARG, "writing %s failed", path);
    return LP_OK;
}

int lp_mlp_load(lp_ctx *ctx, const char *path)
{
    if (!ctx) return fail(LP_ERR_ARG, "ctx is NULL");
    if (!path) return fail(LP_ERR_ARG, "path is NULL");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(LP_ERR_ARG, "cannot open %s", path);
    char magic[8];
    int64_t hdr[2];
    std::vector<float> buf(size_t(NP) * 3);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "LPMLP001", 8) == 0 &&
              std::fread(hdr, 8, 2, f) == 2 && hdr[0] == NP && hdr[1] >= 0 &&
              std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return fail(LP_ERR_ARG, "%s is not a saved network of %lld parameters", path, (long long)NP);
    DeviceGuard dg(ctx->device);
    int rc = alloc_params(ctx);
    if (rc != LP_OK) return rc;
    lpb::MlpState &M = ctx->mlp;
    HIP_TRY(hipMemcpy(M.params.p, buf.data(), size_t(NP) * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(M.adam_m.p, buf.data() + NP, size_t(NP) * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(M.adam_v.p, buf.data() + 2 * NP, size_t(NP) * 4, hipMemcpyHostToDevice));
    HIP_TRY(lpb::launch_cast_params(M.params.as<float>(), M.params16.as<uint16_t>(), NP, nullptr));
    HIP_TRY(hipStreamSynchronize(nullptr));
    M.step = hdr[1];
    M.ready = true;
    return LP_OK;
}

}  // extern "C"
