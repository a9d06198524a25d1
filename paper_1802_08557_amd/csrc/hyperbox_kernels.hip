// hyperbox_kernels.hip -- the closed-form LP over a hyper-rectangle.
//
// For the box [lo_1, hi_1] x ... x [lo_n, hi_n] and a direction l, the maximum
// of l.x over the box is sum_i l_i h_i with h_i = lo_i where l_i < 0 and
// h_i = hi_i otherwise (paper, "Solving a Special Case of LP", Eq. (7)).  No
// simplex is needed; the kernel is a streaming pass over the directions and is
// bound by HBM bandwidth: one thread per direction, whose n-element rows are
// read through the caches in full lines, summed in index order.
#include <stdint.h>

#include "internal.h"

namespace lpb {
namespace {

__global__ __launch_bounds__(256) void hyperbox_kernel(int64_t num, int n, const double *lo, const double *hi,
                                                       const double *l, int shared_box, double *value,
                                                       double *x)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= num) return;
    const double *lk = l + k * n;
    const double *lok = shared_box ? lo : lo + k * n;
    const double *hik = shared_box ? hi : hi + k * n;
    double *xk = x ? x + k * n : nullptr;
    double v = 0.0;
    for (int i = 0; i < n; ++i) {
        const double li = lk[i];
        const double h = (li < 0.0) ? lok[i] : hik[i];
        v = fma(li, h, v);
        if (xk) xk[i] = h;
    }
    value[k] = v;
}

}  // namespace

hipError_t launch_hyperbox(int64_t num, int n, const double *lo, const double *hi, const double *l,
                           int shared_box, double *value, double *x, hipStream_t s)
{
    if (num <= 0) return hipSuccess;
    hipLaunchKernelGGL(hyperbox_kernel, dim3(unsigned((num + 255) / 256)), dim3(256), 0, s, num, n, lo, hi, l,
                       shared_box, value, x);
    return hipGetLastError();
}

}  // namespace lpb
