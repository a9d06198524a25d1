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

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane)
{
    return (uint64_t(1) << lane) - 1;
}

}  // namespace lpb
