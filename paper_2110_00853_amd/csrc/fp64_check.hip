// Accuracy probe of the device FP64 elementary functions (fp64_math.hpp):
// evaluates one of them elementwise over a device array, so that the same
// compiled code the passes inline can be compared with extended-precision
// references on the host.  Built as its own small library; the DG library
// does not export it.
#include <cstdint>

#include "fp64_math.hpp"

namespace {

__global__ void k_fp64_eval(int fn, const double* __restrict__ x, double* __restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = x[i];
    double r;
    switch (fn) {
    case 0: r = cm::frcp(a); break;
    case 1: r = cm::fsqrt(a); break;
    case 2: r = cm::ln_pos(a); break;
    default: r = cm::exp_fin(a); break;
    }
    y[i] = r;
}

}  // namespace

// fn: 0 reciprocal, 1 square root, 2 natural log, 3 exponential.  x, y:
// device arrays of n doubles.  Returns 0, 1 for a bad argument, or the HIP
// error code of the launch.
extern "C" __attribute__((visibility("default"))) int cmx_fp64_eval(int fn, const double* x, double* y, int64_t n,
                                                                    void* stream)
{
    if (fn < 0 || fn > 3 || !x || !y || n < 0) return 1;
    if (n == 0) return 0;
    const int64_t nb = (n + 255) / 256;
    if (nb > 0x7fffffff) return 1;
    hipLaunchKernelGGL(k_fp64_eval, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)stream, fn, x, y, n);
    return (int)hipGetLastError();
}
