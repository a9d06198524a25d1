// device_common.h -- small device helpers shared by the simplex kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpb {

constexpr int kLE = 0, kGE = 1, kEQ = 2;
constexpr int kOptimal = 0, kInfeasible = 1, kUnbounded = 2, kIterLimit = 3, kNumerical = 4,
              kInvalid = 5;
constexpr int kBig = 0x7fffffff;
constexpr int kRowNeg = 1, kRowDead = 8, kRowPad = 16;
// Certificate outcome bits (stats[5]); the values of LP_CERT_* in lpbatch.h.
constexpr int LP_CERT_PRIMAL_OK_BIT = 1, LP_CERT_DUAL_OK_BIT = 2, LP_CERT_RAY_OK_BIT = 4,
              LP_CERT_SINGULAR_BIT = 8, LP_CERT_INFEASIBLE_OK_BIT = 16;

template <typename T> __device__ __forceinline__ T t_inf();
template <> __device__ __forceinline__ float t_inf<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double t_inf<double>() { return __builtin_inf(); }

// Wavefront-uniform read of lane l's value (l must be wavefront-uniform).
__device__ __forceinline__ int lane_get(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_get(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_get(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// A register copy the compiler cannot fold back into its source, so the
// source's register is free for a new load once the copy is made (a value
// prefetched for the next work item can then land where the current one was).
__device__ __forceinline__ double fresh_copy(double v)
{
    double r;
    asm("v_mov_b64 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(v)));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(v >> 32)));
    return int64_t((uint64_t(hi) << 32) | lo);
}
template <typename P>
__device__ __forceinline__ P *uniform_ptr(P *p)
{
    return reinterpret_cast<P *>(uniform64(reinterpret_cast<int64_t>(p)));
}

// Buffer descriptor over `bytes` bytes from p (p wavefront-uniform): the
// hardware range check makes loads at offsets >= bytes return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_over(const void *p, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(const_cast<void *>(p)), short(0), bytes, 0x00020000);
}
__device__ __forceinline__ double buffer_f64(__amdgpu_buffer_rsrc_t rs, int byte_off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, byte_off, 0, 0));
}

// Lexicographic argmin over the wavefront of (k1, k2) carrying p.  Keys are
// unique (k2 is a Bland index) or all invalid, so every lane ends with the
// same winner.
template <typename T>
__device__ __forceinline__ void wave_argmin(T &k1, int &k2, int &p)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const T o1 = __shfl_xor(k1, off);
        const int o2 = __shfl_xor(k2, off);
        const int op = __shfl_xor(p, off);
        if (o1 < k1 || (o1 == k1 && o2 < k2)) { k1 = o1; k2 = o2; p = op; }
    }
}

// The same lexicographic argmin with DPP / permlane reductions instead of
// shuffles through LDS: the least k1, then the least k2 among the lanes that
// hold it, then p from the lowest lane holding both (all 64 lanes active).
template <typename T>
__device__ __forceinline__ void wave_argmin_dpp(T &k1, int &k2, int &p);

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// ---- DPP / permlane reductions (all 64 lanes must be active) ---------------
// Lane patterns (checked on gfx950): quad_perm [1,0,3,2] and [2,3,0,1] swap
// neighbours at distance 1 and 2, row_half_mirror reverses each group of 8,
// row_mirror each row of 16; permlane16_swap(v, v) yields {even-row value,
// odd-row value} and permlane32_swap(v, v) {low-half value, high-half value}
// at the lane's own position.  After the six steps every lane holds the result.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

struct Pair32 { int a, b; };

__device__ __forceinline__ Pair32 swap16(int v)
{
    auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return {int(p[0]), int(p[1])};
}
__device__ __forceinline__ Pair32 swap32(int v)
{
    auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return {int(p[0]), int(p[1])};
}

__device__ __forceinline__ int wave_min_i(int v)
{
    v = min(v, dpp_i<0xB1>(v));
    v = min(v, dpp_i<0x4E>(v));
    v = min(v, dpp_i<0x141>(v));
    v = min(v, dpp_i<0x140>(v));
    Pair32 p = swap16(v);
    v = min(p.a, p.b);
    p = swap32(v);
    return min(p.a, p.b);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f(double v)
{
    return __hiloint2double(dpp_i<CTRL>(__double2hiint(v)), dpp_i<CTRL>(__double2loint(v)));
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}

__device__ __forceinline__ void swap16_f(double v, double &a, double &b)
{
    Pair32 lo = swap16(__double2loint(v)), hi = swap16(__double2hiint(v));
    a = __hiloint2double(hi.a, lo.a);
    b = __hiloint2double(hi.b, lo.b);
}
__device__ __forceinline__ void swap32_f(double v, double &a, double &b)
{
    Pair32 lo = swap32(__double2loint(v)), hi = swap32(__double2hiint(v));
    a = __hiloint2double(hi.a, lo.a);
    b = __hiloint2double(hi.b, lo.b);
}
__device__ __forceinline__ void swap16_f(float v, float &a, float &b)
{
    Pair32 p = swap16(__float_as_int(v));
    a = __int_as_float(p.a);
    b = __int_as_float(p.b);
}
__device__ __forceinline__ void swap32_f(float v, float &a, float &b)
{
    Pair32 p = swap32(__float_as_int(v));
    a = __int_as_float(p.a);
    b = __int_as_float(p.b);
}

// Exact minimum / maximum of a floating-point value over the wavefront (no NaN).
template <typename T>
__device__ __forceinline__ T wave_min_f(T v)
{
    v = fmin(v, dpp_f<0xB1>(v));
    v = fmin(v, dpp_f<0x4E>(v));
    v = fmin(v, dpp_f<0x141>(v));
    v = fmin(v, dpp_f<0x140>(v));
    T a, b;
    swap16_f(v, a, b);
    v = fmin(a, b);
    swap32_f(v, a, b);
    return fmin(a, b);
}
template <typename T>
__device__ __forceinline__ T wave_max_f(T v)
{
    v = fmax(v, dpp_f<0xB1>(v));
    v = fmax(v, dpp_f<0x4E>(v));
    v = fmax(v, dpp_f<0x141>(v));
    v = fmax(v, dpp_f<0x140>(v));
    T a, b;
    swap16_f(v, a, b);
    v = fmax(a, b);
    swap32_f(v, a, b);
    return fmax(a, b);
}

template <typename T>
__device__ __forceinline__ void wave_argmin_dpp(T &k1, int &k2, int &p)
{
    const T best = wave_min_f(k1);
    const bool tie = k1 == best;
    const int kmin = wave_min_i(tie ? k2 : kBig);
    const uint64_t win = __ballot(tie && k2 == kmin);
    const int src = win ? __builtin_ctzll(win) : 0;
    k1 = best;
    k2 = kmin;
    p = lane_get(p, src);
}

// Called once per workgroup (one thread) when it leaves its work loop: the
// last workgroup to finish returns the launch's counters to 0 for the next
// launch on the stream.  Every queue atomic of a workgroup has returned
// before it gets here (its result decides the loop exit).
__device__ __forceinline__ void finish_launch(int32_t *queue, int32_t *done, int32_t *extra)
{
    const int fin = atomicAdd(done, 1);
    if (fin == int(gridDim.x) - 1) {
        atomicExch(queue, 0);
        atomicExch(done, 0);
        if (extra) atomicExch(extra, 0);
    }
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane)
{
    return (uint64_t(1) << lane) - 1;
}

}  // namespace lpb
