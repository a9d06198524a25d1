// scale_kernels.hip -- optional geometric-mean scaling with power-of-two factors.
//
// The paper's method pivots on the LP as given (Sec. 4 builds the tableau from
// A, b and c directly).  Badly scaled constraint rows and columns hurt the
// single-precision tableau most, so the library can precondition a batch first:
// row factors 2^r_i and column factors 2^s_j, chosen on binary exponents
// E_ij = floor(log2 |a_ij|) of the finite non-zero entries.  Each pass sets
//     r_i = -floor((max_j (E_ij + s_j) + min_j (E_ij + s_j) + 1) / 2)
// for every row with entries, then s_j the same way over the column with the
// new r_i (rows / columns without entries keep 0, every exponent is clamped to
// [-128, 128]).  The scaled LP a'_ij = a_ij 2^(r_i + s_j), b'_i = b_i 2^r_i,
// c'_j = c_j 2^s_j has exactly the original feasible set under x_j = x'_j 2^s_j
// and the same objective values: multiplying by a power of two rounds nothing.
// All exponent work is integer arithmetic, so the factors are the same on every
// machine and in every order of evaluation.
//
// Small LPs (at most 8192 entries, 2048 rows + columns, and an LDS region of
// at most 16 KB) take one wavefront each, with no barrier: the exponents are
// staged once into the wavefront's LDS region as int16, row-major with an odd
// number of 32-bit words per row (so lanes walking different rows of one
// column hit different banks); a row sweep gives lane i row i (it loops over
// the row's columns), a column sweep lane j column j; the factors live in LDS
// next to the exponents.  A is read twice in all: to stage the exponents and
// to write A'.  Larger LPs take a 256-thread workgroup each: a wavefront per
// row with lanes across the row, a thread per column walking down the rows,
// exponents recomputed from A in every sweep and the factors kept in the
// output arrays.

#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "internal.h"

namespace lpb {
namespace {

constexpr int kThreads = 256;
constexpr int kStageE = 8192;
constexpr int kStageRS = 2048;
constexpr int kWaveRegionMax = 16384;
constexpr int kUnroll = 8;  // loads per lane in flight in the wavefront kernel's sweeps over A
constexpr int kAbsent = -32768;  // exponent marker of a zero or non-finite entry
constexpr int kExpCap = 128;

__device__ __forceinline__ int binary_exponent(double v)
{
    if (v == 0.0 || !isfinite(v)) return kAbsent;
    int e;
    (void)frexp(v, &e);
    return e - 1;
}

// -floor((hi + lo + 1) / 2), clamped; 0 when no entry took part (hi < lo).
__device__ __forceinline__ int midpoint_exponent(int hi, int lo)
{
    if (hi < lo) return 0;
    const int e = -((hi + lo + 1) >> 1);
    return e < -kExpCap ? -kExpCap : (e > kExpCap ? kExpCap : e);
}

__device__ __forceinline__ int wave_max_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_min_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

struct ScaleArgs {
    int64_t num;
    int32_t um, un;  // uniform shape, or 0 with the arrays below
    const int32_t *m, *n;
    const int64_t *aoff, *roff, *coff;
    int32_t passes;
    const double *A, *b, *c;
    double *A_out, *b_out, *c_out;
    int32_t *rexp, *cexp;
    int32_t region;  // LDS bytes per wavefront of the wavefront kernel (0: not launched)
};

// Row stride (int16 elements) of the staged exponents: n rounded up to an odd
// number of 32-bit words.
__host__ __device__ __forceinline__ int exp_ld(int n)
{
    const int w = (n + 1) >> 1;
    return 2 * (w | 1);
}

__host__ __device__ __forceinline__ int64_t wave_region(int m, int n)
{
    return ((2 * int64_t(m) * exp_ld(n) + 15) & ~int64_t(15)) + ((4 * int64_t(m + n) + 15) & ~int64_t(15));
}

// LPs the wavefront kernel takes; the workgroup kernel takes the others.
__device__ __forceinline__ bool wave_takes(const ScaleArgs &a, int m, int n)
{
    return a.region > 0 && int64_t(m) * n <= kStageE && m + n <= kStageRS && wave_region(m, n) <= a.region;
}

struct LpGeom {
    int m, n;
    int64_t ao, ro, co;
};

__device__ __forceinline__ LpGeom geom(const ScaleArgs &a, int64_t k)
{
    LpGeom g;
    g.m = a.um ? a.um : a.m[k];
    g.n = a.un ? a.un : a.n[k];
    g.ao = a.um ? k * int64_t(g.m) * g.n : a.aoff[k];
    g.ro = a.um ? k * int64_t(g.m) : a.roff[k];
    g.co = a.un ? k * int64_t(g.n) : a.coff[k];
    return g;
}

// Writes b', c' and the exponents of one LP; t / T: this thread's index and
// the number of threads sharing the LP.
__device__ __forceinline__ void write_vectors(const ScaleArgs &a, const LpGeom &g, const int *r, const int *s, int t,
                                              int T)
{
    for (int i = t; i < g.m; i += T) {
        a.b_out[g.ro + i] = ldexp(a.b[g.ro + i], r[i]);
        a.rexp[g.ro + i] = r[i];
    }
    for (int j = t; j < g.n; j += T) {
        if (a.c_out) a.c_out[g.co + j] = ldexp(a.c[g.co + j], s[j]);
        a.cexp[g.co + j] = s[j];
    }
}

// The passes of one LP.  E(i, j) gives the exponent of entry (i, j); r and s
// are the factor exponents (LDS or the output arrays).
template <typename EFn>
__device__ void scale_passes(int mk, int nk, int passes, EFn E, int *r, int *s)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kBig = 1 << 20;
    for (int j = threadIdx.x; j < nk; j += kThreads) s[j] = 0;
    __syncthreads();
    for (int p = 0; p < passes; ++p) {
        for (int i = wave; i < mk; i += kThreads / 64) {
            int hi = -kBig, lo = kBig;
            for (int j = lane; j < nk; j += 64) {
                const int e = E(i, j);
                if (e != kAbsent) {
                    hi = max(hi, e + s[j]);
                    lo = min(lo, e + s[j]);
                }
            }
            hi = wave_max_i(hi);
            lo = wave_min_i(lo);
            if (lane == 0) r[i] = midpoint_exponent(hi, lo);
        }
        __syncthreads();
        for (int j = threadIdx.x; j < nk; j += kThreads) {
            int hi = -kBig, lo = kBig;
            for (int i = 0; i < mk; ++i) {
                const int e = E(i, j);
                if (e != kAbsent) {
                    hi = max(hi, e + r[i]);
                    lo = min(lo, e + r[i]);
                }
            }
            s[j] = midpoint_exponent(hi, lo);
        }
        __syncthreads();
    }
    if (passes == 0) {
        for (int i = threadIdx.x; i < mk; i += kThreads) r[i] = 0;
        __syncthreads();
    }
}

// One wavefront per small LP (see above).
__global__ __launch_bounds__(kThreads) void scale_wave_kernel(ScaleArgs a)
{
    extern __shared__ __align__(16) char lds[];
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    char *region = lds + (threadIdx.x >> 6) * a.region;
    constexpr int kBig = 1 << 20;
    for (int64_t k = int64_t(blockIdx.x) * wpb + (threadIdx.x >> 6); k < a.num; k += int64_t(gridDim.x) * wpb) {
        const LpGeom g = geom(a, k);
        if (!wave_takes(a, g.m, g.n)) continue;
        const int ld = exp_ld(g.n);
        int16_t *E = reinterpret_cast<int16_t *>(region);
        int *r = reinterpret_cast<int *>(region + ((2 * g.m * ld + 15) & ~15));
        int *s = r + g.m;
        const double *Ak = a.A + g.ao;
        const int mn = g.m * g.n;
        // Flat element order, eight loads per lane in flight before the first
        // is used.
        for (int f0 = 0; f0 < mn; f0 += 64 * kUnroll) {
            double v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int f = f0 + u * 64 + lane;
                v[u] = f < mn ? Ak[f] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int f = f0 + u * 64 + lane;
                if (f < mn) {
                    const int i = f / g.n, j = f - i * g.n;
                    E[i * ld + j] = int16_t(binary_exponent(v[u]));
                }
            }
        }
        for (int j = lane; j < g.n; j += 64) s[j] = 0;
        for (int i = lane; i < g.m; i += 64) r[i] = 0;
        // A wavefront's LDS accesses complete in program order; the barrier
        // only keeps the compiler from moving them across the sweeps.
        __builtin_amdgcn_wave_barrier();
        for (int p = 0; p < a.passes; ++p) {
            for (int i = lane; i < g.m; i += 64) {
                int hi = -kBig, lo = kBig;
                const int16_t *Ei = E + i * ld;
#pragma unroll 8
                for (int j = 0; j < g.n; ++j) {
                    const int e = Ei[j];
                    const int v = e + s[j];
                    hi = e != kAbsent ? max(hi, v) : hi;
                    lo = e != kAbsent ? min(lo, v) : lo;
                }
                r[i] = midpoint_exponent(hi, lo);
            }
            __builtin_amdgcn_wave_barrier();
            for (int j = lane; j < g.n; j += 64) {
                int hi = -kBig, lo = kBig;
#pragma unroll 8
                for (int i = 0; i < g.m; ++i) {
                    const int e = E[i * ld + j];
                    const int v = e + r[i];
                    hi = e != kAbsent ? max(hi, v) : hi;
                    lo = e != kAbsent ? min(lo, v) : lo;
                }
                s[j] = midpoint_exponent(hi, lo);
            }
            __builtin_amdgcn_wave_barrier();
        }
        double *Ao = a.A_out + g.ao;
        for (int f0 = 0; f0 < mn; f0 += 64 * kUnroll) {
            double v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int f = f0 + u * 64 + lane;
                v[u] = f < mn ? Ak[f] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int f = f0 + u * 64 + lane;
                if (f < mn) {
                    const int i = f / g.n, j = f - i * g.n;
                    Ao[f] = ldexp(v[u], r[i] + s[j]);
                }
            }
        }
        write_vectors(a, g, r, s, lane, 64);
        __builtin_amdgcn_wave_barrier();  // the region is reused by the next LP
    }
}

// One workgroup per LP the wavefront kernel does not take.
__global__ __launch_bounds__(kThreads) void scale_kernel(ScaleArgs a)
{
    for (int64_t k = blockIdx.x; k < a.num; k += gridDim.x) {
        const LpGeom g = geom(a, k);
        if (wave_takes(a, g.m, g.n)) continue;
        const double *Ak = a.A + g.ao;
        int *r = a.rexp + g.ro, *s = a.cexp + g.co;
        scale_passes(g.m, g.n, a.passes, [&](int i, int j) { return binary_exponent(Ak[int64_t(i) * g.n + j]); }, r,
                     s);
        double *Ao = a.A_out + g.ao;
        for (int i = 0; i < g.m; ++i) {
            const int ri = r[i];
            for (int j = threadIdx.x; j < g.n; j += kThreads)
                Ao[int64_t(i) * g.n + j] = ldexp(Ak[int64_t(i) * g.n + j], ri + s[j]);
        }
        write_vectors(a, g, r, s, threadIdx.x, kThreads);
        __syncthreads();
    }
}

// out[i] = in[i] * 2^e[i] (period 0), or 2^e[i % period].
__global__ __launch_bounds__(256) void ldexp_kernel(int64_t count, const double *in, const int32_t *e,
                                                    int64_t period, double *out)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * blockDim.x)
        out[i] = ldexp(in[i], e[period ? i % period : i]);
}

}  // namespace

hipError_t launch_scale(int64_t num, int32_t um, int32_t un, const int32_t *m, const int32_t *n,
                        const int64_t *aoff, const int64_t *roff, const int64_t *coff, const int32_t *host_m,
                        const int32_t *host_n, int32_t passes, const double *A, const double *b, const double *c,
                        double *A_out, double *b_out, double *c_out, int32_t *rexp, int32_t *cexp, hipStream_t s)
{
    if (num <= 0) return hipSuccess;
    // The wavefront kernel's region fits the largest LP it takes; the others
    // go to the workgroup kernel (the kernels test the same predicate).
    int64_t region = 0;
    bool any_large = false;
    for (int64_t k = 0; k < (um ? 1 : num); ++k) {
        const int mk = um ? um : host_m[k], nk = un ? un : host_n[k];
        const int64_t rg = wave_region(mk, nk);
        if (int64_t(mk) * nk <= kStageE && mk + nk <= kStageRS && rg <= kWaveRegionMax)
            region = std::max(region, rg);
        else
            any_large = true;
    }
    ScaleArgs a{num, um, un, m, n, aoff, roff, coff, passes, A, b, c, A_out, b_out, c_out, rexp, cexp,
                int32_t(region)};
    if (region > 0) {
        constexpr int wpb = 4;  // 4 regions of at most 16 KB
        const int64_t blocks = std::min<int64_t>((num + wpb - 1) / wpb, 32768);
        hipLaunchKernelGGL(scale_wave_kernel, dim3(unsigned(blocks)), dim3(64 * wpb), size_t(wpb) * region, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (any_large) {
        hipLaunchKernelGGL(scale_kernel, dim3(unsigned(num < 16384 ? num : 16384)), dim3(kThreads), 0, s, a);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_ldexp(int64_t count, const double *in, const int32_t *e, int64_t period, double *out,
                        hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(ldexp_kernel, dim3(unsigned(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, count, in,
                       e, period, out);
    return hipGetLastError();
}

}  // namespace lpb
