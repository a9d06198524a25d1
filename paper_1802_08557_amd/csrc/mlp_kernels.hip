// mlp_kernels.hip -- the warm-start scoring network (20 -> 256 -> 256 -> 120,
// ReLU) on the matrix cores: BF16 operands, FP32 accumulation.
//
// Every layer, forward and backward, is one launch of a strided GEMM
//     C[i][j] = sum_k A(i, k) B(k, j),  A(i, k) = a[i*sai + k*sak],
//                                        B(k, j) = b[k*sbk + j*sbj]
// on v_mfma_f32_16x16x16_bf16 tiles, one wavefront per 32 x 32 block of C,
// followed by a fused epilogue (bias, ReLU mask of the forward activation,
// FP32 and/or rounded BF16 stores).  The products are small (the widest is
// 256 x 256), so one strided kernel serves the six backward shapes too; the
// forward reads both operands along k with 8-byte loads.
//
// The remaining kernels are elementwise or row-wise: FP32 -> BF16 input
// conversion, the logistic loss and its gradient, bias gradients (column sums
// in a fixed order), AdamW on the FP32 master weights with a fresh BF16 copy,
// and the per-direction top-k of the scores.  Every reduction runs in a fixed
// order, so a training step is deterministic.
#include <math.h>
#include <stdint.h>

#include "internal.h"

namespace lpb {
namespace {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> bfloat16 bits, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

// Four consecutive-k operand values of row (or column) r, k = k0 .. k0 + 3;
// zero outside [0, R) x [0, K).
__device__ __forceinline__ s16x4 load_frag(const uint16_t *p, int r, int R, int64_t sr, int k0, int K,
                                           int64_t sk)
{
    s16x4 v = {0, 0, 0, 0};
    if (r >= R) return v;
    const uint16_t *q = p + int64_t(r) * sr;
    if (sk == 1 && k0 + 3 < K && ((int64_t(r) * sr + k0) & 3) == 0) {
        const uint2 w = *reinterpret_cast<const uint2 *>(q + k0);
        v[0] = short(w.x & 0xFFFF);
        v[1] = short(w.x >> 16);
        v[2] = short(w.y & 0xFFFF);
        v[3] = short(w.y >> 16);
        return v;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (k0 + t < K) v[t] = short(q[int64_t(k0 + t) * sk]);
    return v;
}

__global__ __launch_bounds__(64) void gemm_bf16_kernel(MlpGemm g)
{
    const int lane = threadIdx.x;
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int r16 = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        // A fragment: row i0 + 16 a + (lane % 16), k = k0 + 4 (lane / 16) + t;
        // B fragment: column j0 + 16 b + (lane % 16), same k.
        s16x4 fa[2], fb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) fa[a] = load_frag(g.a, i0 + 16 * a + r16, g.M, g.sai, k0 + kq, g.K, g.sak);
#pragma unroll
        for (int b = 0; b < 2; ++b) fb[b] = load_frag(g.b, j0 + 16 * b + r16, g.N, g.sbj, k0 + kq, g.K, g.sbk);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    // D layout: lane holds column (lane % 16), rows 4 (lane / 16) + t.
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int j = j0 + 16 * b + r16;
            if (j >= g.N) continue;
            const float bj = g.bias ? g.bias[j] : 0.f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = i0 + 16 * a + kq + t;
                if (i >= g.M) continue;
                float v = acc[a][b][t] + bj;
                const int64_t o = int64_t(i) * g.ldc + j;
                if (g.mask && !(g.mask[o] > 0.f)) v = 0.f;
                if (g.c32) g.c32[o] = v;
                if (g.c16) g.c16[o] = to_bf16(g.relu ? fmaxf(v, 0.f) : v);
            }
        }
}

__global__ void to_bf16_kernel(const float *x, uint16_t *y, int64_t count)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) y[i] = to_bf16(x[i]);
}

// dS = (sigmoid(S) - Y) / (B * O) in FP32 and BF16; row_loss[b] = sum over the
// row of softplus(S) - Y S (summed in column order).
__global__ __launch_bounds__(256) void bce_kernel(const float *S, const uint8_t *Y, int64_t B, int O, float *dS,
                                                  uint16_t *dS16, float *row_loss)
{
    // One wavefront per row: lane j takes outputs j, j + 64, ...; the row's
    // loss is reduced over the lanes by a fixed butterfly.
    const int lane = threadIdx.x & 63;
    const int64_t b = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (b >= B) return;
    const float inv = 1.0f / (float(B) * float(O));
    float acc = 0.f;
    for (int j = lane; j < O; j += 64) {
        const int64_t o = b * O + j;
        const float s = S[o];
        const float y = Y[o] ? 1.f : 0.f;
        const float sp = fmaxf(s, 0.f) + log1pf(expf(-fabsf(s)));
        acc += sp - y * s;
        const float sg = 1.f / (1.f + expf(-s));
        const float d = (sg - y) * inv;
        dS[o] = d;
        dS16[o] = to_bf16(d);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) row_loss[b] = acc;
}

// Mean of the row losses, one workgroup, fixed order: each thread sums a
// strided slice, then a tree over the threads.
__global__ __launch_bounds__(256) void mean_kernel(const float *row_loss, int64_t B, int O, float *out)
{
    __shared__ double part[256];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < B; b += 256) s += double(row_loss[b]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = float(part[0] / (double(B) * O));
}

// db[j] = sum_b dZ[b][j]: 64 columns per workgroup; thread (c, p) sums rows
// p, p + 16, ... of column c in order, then the sixteen partial sums are added
// in order of p.
__global__ __launch_bounds__(1024) void colsum_kernel(const float *dZ, int64_t B, int N, float *db)
{
    __shared__ float part[16][64];
    const int c = threadIdx.x & 63, p = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    float s = 0.f;
    if (j < N)
        for (int64_t b = p; b < B; b += 16) s += dZ[b * N + j];
    part[p][c] = s;
    __syncthreads();
    if (p == 0 && j < N) {
        float t = part[0][c];
#pragma unroll
        for (int q = 1; q < 16; ++q) t += part[q][c];
        db[j] = t;
    }
}

// AdamW on the FP32 master copy; decay[i] = 1 for weights, 0 for biases.
__global__ void adamw_kernel(float *w, const float *g, float *m, float *v, uint16_t *w16, int64_t count,
                             MlpAdam h, int64_t decay_lo0, int64_t decay_hi0, int64_t decay_lo1,
                             int64_t decay_hi1, int64_t decay_lo2, int64_t decay_hi2)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const bool decay = (i >= decay_lo0 && i < decay_hi0) || (i >= decay_lo1 && i < decay_hi1) ||
                       (i >= decay_lo2 && i < decay_hi2);
    const float gi = g[i];
    const float mi = h.beta1 * m[i] + (1.f - h.beta1) * gi;
    const float vi = h.beta2 * v[i] + (1.f - h.beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mhat = mi / h.bc1;
    const float vhat = vi / h.bc2;
    float wi = w[i];
    wi = wi - h.lr * mhat / (sqrtf(vhat) + h.eps) - (decay ? h.lr * h.wd * w[i] : 0.f);
    w[i] = wi;
    w16[i] = to_bf16(wi);
}

__global__ void cast_params_kernel(const float *w, uint16_t *w16, int64_t count)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) w16[i] = to_bf16(w[i]);
}

// Top-k of each row of S [B][O] (O <= 128): one wavefront per row; the entry
// of rank r (number of entries that are larger, or equal with a lower index)
// goes to out[b][r] when r < k.
__global__ __launch_bounds__(64) void topk_kernel(const float *S, int64_t B, int O, int k, int32_t *out)
{
    const int64_t b = blockIdx.x;
    if (b >= B) return;
    __shared__ float s[128];
    const int lane = threadIdx.x;
    for (int j = lane; j < O; j += 64) s[j] = S[b * O + j];
    __syncthreads();
    for (int j = lane; j < O; j += 64) {
        const float v = s[j];
        int r = 0;
        for (int t = 0; t < O; ++t) {
            const float u = s[t];
            r += (u > v || (u == v && t < j)) ? 1 : 0;
        }
        if (r < k) out[b * k + r] = j;
    }
}


// ---- Fused inference --------------------------------------------------------
// All three layers and the top-k for a tile of 64 directions in one workgroup
// of four wavefronts: the input tile and both hidden activations stay in LDS
// (BF16), the weights stream from L2 as MFMA fragments.  The products, their
// k order and the epilogues are those of gemm_bf16_kernel, so the scores are
// the same bits as the layer-by-layer path.

// ---- Top-k by a bitonic sort over the wavefront ------------------------------
// Key of entry t with score v: the score's bits mapped to an order-preserving
// unsigned integer (-0 taken as +0, so equal scores give equal keys) above
// 127 - t, so that descending key order is descending score with equal scores
// in ascending entry order.
__device__ __forceinline__ uint64_t topk_key(float v, int t)
{
    const uint32_t u = __float_as_uint(v + 0.0f);
    const uint32_t mono = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return (uint64_t(mono) << 32) | uint32_t(127 - t);
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, 0xf, 0xf, false));
}

// Value of lane (lane ^ J).  DPP patterns: quad_perm [1,0,3,2] (0xB1) and
// [2,3,0,1] (0x4E) swap at distance 1 and 2; [3,2,1,0] (0x1B) after
// row_half_mirror (0x141, i -> i ^ 7 in each group of 8) gives i ^ 4;
// row_half_mirror after row_mirror (0x140, i -> i ^ 15 in each row of 16) gives
// i ^ 8; the permlane swaps exchange rows (16) and halves (32).
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v)
{
    const int lane = threadIdx.x & 63;
    if constexpr (J == 1) return dpp32<0xB1>(v);
    else if constexpr (J == 2) return dpp32<0x4E>(v);
    else if constexpr (J == 4) return dpp32<0x1B>(dpp32<0x141>(v));
    else if constexpr (J == 8) return dpp32<0x141>(dpp32<0x140>(v));
    else if constexpr (J == 16) {
        auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return ((lane >> 4) & 1) ? uint32_t(p[0]) : uint32_t(p[1]);
    } else {
        auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane >> 5) ? uint32_t(p[0]) : uint32_t(p[1]);
    }
}

template <int J>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v)
{
    return (uint64_t(xor_lane<J>(uint32_t(v >> 32))) << 32) | xor_lane<J>(uint32_t(v));
}

// One compare-exchange step (block size SZ, distance J < 64) on both halves:
// element e keeps the larger key when bit J of e is clear exactly when bit SZ
// of e is clear (descending blocks), the smaller otherwise.
template <int SZ, int J>
__device__ __forceinline__ void bitonic_step(uint64_t &k0, uint64_t &k1)
{
    const int lane = threadIdx.x & 63;
    const uint64_t p0 = xor_lane64<J>(k0), p1 = xor_lane64<J>(k1);
    const bool lower = (lane & J) == 0;
    const bool up0 = ((lane + 0) & SZ) == 0, up1 = ((lane + 64) & SZ) == 0;
    const bool max0 = lower == up0, max1 = lower == up1;
    // Take the partner's key when it is larger and this element keeps the
    // larger, or it is not larger and this element keeps the smaller.
    k0 = ((p0 > k0) == max0) ? p0 : k0;
    k1 = ((p1 > k1) == max1) ? p1 : k1;
}

template <int SZ, int J>
__device__ __forceinline__ void bitonic_merge2(uint64_t &a0, uint64_t &a1, uint64_t &b0, uint64_t &b1)
{
    if constexpr (J == 64) {
        const uint64_t ah = a0 > a1 ? a0 : a1, al = a0 > a1 ? a1 : a0;
        const uint64_t bh = b0 > b1 ? b0 : b1, bl = b0 > b1 ? b1 : b0;
        a0 = ah; a1 = al; b0 = bh; b1 = bl;
    } else {
        bitonic_step<SZ, J>(a0, a1);
        bitonic_step<SZ, J>(b0, b1);
    }
    if constexpr (J > 1) bitonic_merge2<SZ, J / 2>(a0, a1, b0, b1);
}

template <int SZ>
__device__ __forceinline__ void bitonic_stage2(uint64_t &a0, uint64_t &a1, uint64_t &b0, uint64_t &b1)
{
    bitonic_merge2<SZ, SZ / 2>(a0, a1, b0, b1);
    if constexpr (SZ < 128) bitonic_stage2<SZ * 2>(a0, a1, b0, b1);
}

// Sorts two independent sets of 128 keys, (a0, a1) and (b0, b1), each in
// descending order over positions lane (x0) and lane + 64 (x1); all 64
// lanes must be active.
__device__ __forceinline__ void bitonic_desc128x2(uint64_t &a0, uint64_t &a1, uint64_t &b0, uint64_t &b1)
{
    bitonic_stage2<2>(a0, a1, b0, b1);
}

constexpr int kTile = 64;
constexpr int kIn = 20, kHid = 256, kOut = 120;
constexpr int64_t kOW1 = 0, kOB1 = kOW1 + int64_t(kHid) * kIn, kOW2 = kOB1 + kHid,
                  kOB2 = kOW2 + int64_t(kHid) * kHid, kOW3 = kOB2 + kHid, kOB3 = kOW3 + int64_t(kOut) * kHid;

// Row strides (BF16 elements) of the LDS tiles, padded so that the sixteen
// rows one MFMA fragment load touches fall in different LDS banks.
constexpr int kLdx = 40, kLdh = kHid + 8;

__host__ __device__ constexpr int64_t infer_lds_bytes()
{
    return int64_t(kTile) * kLdx * 2 + 2 * int64_t(kTile) * kLdh * 2;
}

// Weight fragment: row n of a [rows][K] BF16 matrix, k = k0 .. k0+3 (zero past K or rows).
__device__ __forceinline__ s16x4 wfrag(const uint16_t *w, int n, int rows, int K, int k0)
{
    s16x4 v = {0, 0, 0, 0};
    if (n >= rows) return v;
    if (k0 + 3 < K) {
        const uint2 q = *reinterpret_cast<const uint2 *>(w + int64_t(n) * K + k0);
        v[0] = short(q.x & 0xFFFF);
        v[1] = short(q.x >> 16);
        v[2] = short(q.y & 0xFFFF);
        v[3] = short(q.y >> 16);
        return v;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (k0 + t < K) v[t] = short(w[int64_t(n) * K + k0 + t]);
    return v;
}

// One layer on the tile: out[64][NT*16*4 waves] = act[64][K] * W^T (+ bias),
// this wavefront taking N tiles NT*wave .. NT*wave + NT-1.  Epilogue: BF16
// ReLU activations (h16, row stride kLdh) or FP32 scores (s32, row stride 128).
template <int NT>
__device__ __forceinline__ void tile_layer(const uint16_t *act, int lda, int K, const uint16_t *w, int rows,
                                           const float *bias, uint16_t *h16, float *s32)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc[4][NT];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[a][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // Weight fragments are loaded one k step ahead of their use.
    s16x4 fbn[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) fbn[j] = wfrag(w, (NT * wave + j) * 16 + r16, rows, K, kq);
    for (int k0 = 0; k0 < K; k0 += 16) {
        s16x4 fa[4], fb[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) fb[j] = fbn[j];
        if (k0 + 16 < K) {
#pragma unroll
            for (int j = 0; j < NT; ++j) fbn[j] = wfrag(w, (NT * wave + j) * 16 + r16, rows, K, k0 + 16 + kq);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) fa[a] = *reinterpret_cast<const s16x4 *>(act + (16 * a + r16) * lda + k0 + kq);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[a][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[j], acc[a][j], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int col = (NT * wave + j) * 16 + r16;
            const float bj = col < rows ? bias[col] : 0.f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int row = 16 * a + kq + t;
                const float v = acc[a][j][t] + bj;
                if (h16) h16[row * kLdh + col] = to_bf16(fmaxf(v, 0.f));
                else s32[row * 128 + col] = v;
            }
        }
}

__global__ __launch_bounds__(256) void mlp_infer_kernel(const float *dirs, int64_t B, const uint16_t *w16,
                                                        const float *w32, float *scores, int32_t *topk, int k)
{
    extern __shared__ __align__(16) char smem[];
    uint16_t *x16 = reinterpret_cast<uint16_t *>(smem);                         // [64][kLdx]
    uint16_t *h1 = reinterpret_cast<uint16_t *>(smem + kTile * kLdx * 2);       // [64][kLdh]
    uint16_t *h2 = h1 + kTile * kLdh;                                             // [64][kLdh]
    float *sc = reinterpret_cast<float *>(h1);                                    // [64][128], after layer 2
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t b0 = int64_t(blockIdx.x) * kTile;
    for (int e = tid; e < kTile * 32; e += 256) {
        const int r = e >> 5, kk = e & 31;
        const int64_t b = b0 + r;
        x16[r * kLdx + kk] = to_bf16((b < B && kk < kIn) ? dirs[b * kIn + kk] : 0.f);
    }
    __syncthreads();
    tile_layer<4>(x16, kLdx, kIn, w16 + kOW1, kHid, w32 + kOB1, h1, nullptr);
    __syncthreads();
    tile_layer<4>(h1, kLdh, kHid, w16 + kOW2, kHid, w32 + kOB2, h2, nullptr);
    __syncthreads();
    tile_layer<2>(h2, kLdh, kHid, w16 + kOW3, kOut, w32 + kOB3, nullptr, sc);
    __syncthreads();
    // Scores out, and the top-k of every row by rank counting (one wavefront
    // per sixteen rows; lanes hold entries lane and lane + 64).
    // Two rows per step, so that the two sorts' independent instruction
    // chains interleave.
    for (int rr = 0; rr < kTile / 4; rr += 2) {
        const int row = wave * (kTile / 4) + rr;
        const int64_t b = b0 + row;
        if (b >= B) break;
        const bool two = b + 1 < B;
        float s0[2], s1[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            s0[q] = sc[(row + q) * 128 + lane];
            s1[q] = (lane + 64 < kOut) ? sc[(row + q) * 128 + lane + 64] : 0.f;
        }
        if (scores) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                if (q == 1 && !two) break;
                scores[(b + q) * kOut + lane] = s0[q];
                if (lane + 64 < kOut) scores[(b + q) * kOut + lane + 64] = s1[q];
            }
        }
        if (topk) {
            // Sort each row's 120 keys (and 8 padding keys below every real
            // one) in descending order; position e = lane + 64 h then holds
            // the entry of rank e.
            uint64_t ka0 = topk_key(s0[0], lane), kb0 = topk_key(s0[1], lane);
            uint64_t ka1 = (lane + 64 < kOut) ? topk_key(s1[0], lane + 64) : 0;
            uint64_t kb1 = (lane + 64 < kOut) ? topk_key(s1[1], lane + 64) : 0;
            bitonic_desc128x2(ka0, ka1, kb0, kb1);
            if (lane < k) topk[b * k + lane] = 127 - int(uint32_t(ka0));
            if (lane + 64 < k) topk[b * k + lane + 64] = 127 - int(uint32_t(ka1));
            if (two) {
                if (lane < k) topk[(b + 1) * k + lane] = 127 - int(uint32_t(kb0));
                if (lane + 64 < k) topk[(b + 1) * k + lane + 64] = 127 - int(uint32_t(kb1));
            }
        }
    }
}

}  // namespace

hipError_t launch_mlp_gemm(const MlpGemm &g, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    dim3 grid((g.M + 31) / 32, (g.N + 31) / 32);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(64), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *x, uint16_t *y, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, x, y, count);
    return hipGetLastError();
}

hipError_t launch_bce(const float *S, const uint8_t *Y, int64_t B, int O, float *dS, uint16_t *dS16,
                      float *row_loss, float *loss, hipStream_t s)
{
    hipLaunchKernelGGL(bce_kernel, dim3(unsigned((B + 3) / 4)), dim3(256), 0, s, S, Y, B, O, dS, dS16, row_loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, s, row_loss, B, O, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *dZ, int64_t B, int N, float *db, hipStream_t s)
{
    hipLaunchKernelGGL(colsum_kernel, dim3(unsigned((N + 63) / 64)), dim3(1024), 0, s, dZ, B, N, db);
    return hipGetLastError();
}

hipError_t launch_adamw(float *w, const float *g, float *m, float *v, uint16_t *w16, int64_t count,
                        const MlpAdam &h, const int64_t (&decay)[6], hipStream_t s)
{
    hipLaunchKernelGGL(adamw_kernel, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, w, g, m, v, w16,
                       count, h, decay[0], decay[1], decay[2], decay[3], decay[4], decay[5]);
    return hipGetLastError();
}

hipError_t launch_cast_params(const float *w, uint16_t *w16, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(cast_params_kernel, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, w, w16, count);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const float *dirs, int64_t B, const uint16_t *w16, const float *w32, float *scores,
                            int32_t *topk, int k, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_infer_kernel, dim3(unsigned((B + kTile - 1) / kTile)), dim3(256), size_t(infer_lds_bytes()), s,
                       dirs, B, w16, w32, scores, topk, k);
    return hipGetLastError();
}

hipError_t mlp_configure()
{
    return hipFuncSetAttribute((const void *)mlp_infer_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(infer_lds_bytes()));
}

hipError_t launch_topk(const float *S, int64_t B, int O, int k, int32_t *out, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(topk_kernel, dim3(unsigned(B)), dim3(64), 0, s, S, B, O, k, out);
    return hipGetLastError();
}

}  // namespace lpb
