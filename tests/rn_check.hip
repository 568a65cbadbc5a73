// rn_check.hip -- test helper: runs the rounded-to-nearest sequences of the
// Euler kernels (paper_1811_08282_amd/csrc/rn_ops.h) on device arrays, for
// tests/test_gpu_rn_ops.py to compare with IEEE division and square root.
// Built into tests/librn_check.so by the build step.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../paper_1811_08282_amd/csrc/rn_ops.h"

namespace {

// out[6 i + ..]: limiter(a), sqrt(a), a / d, c / d (second quotient by d),
// sqrt of the pair (a, c) taken together: sqrt(a), sqrt(c)
__global__ void k_rn_check(const double *a, const double *c, const double *d, double *out,
                           int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double x = a[i], y = c[i], z = d[i];
    double *o = out + 6 * i;
    o[0] = sw::limiter(x);
    double s0, s1;
    sw::rn_sqrt2(x, x, s0, s1);
    o[1] = s0;
    sw::RnDiv dv;
    o[2] = sw::rn_div_keep(x, z, dv);
    o[3] = sw::rn_div_again(y, dv);
    sw::rn_sqrt2(x, y, o[4], o[5]);
}

} // namespace

// n values each in device arrays a, c, d; out holds 6 n doubles.  Returns a
// hipError_t value (0 on success); synchronises the device.
extern "C" int rn_check(const double *a, const double *c, const double *d, double *out, int64_t n)
{
    if (n <= 0)
        return 0;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_rn_check, dim3(blocks), dim3(256), 0, 0, a, c, d, out, n);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    return (int)e;
}
