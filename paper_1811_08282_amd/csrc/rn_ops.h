// rn_ops.h -- binary64 division, square root and limiter clamp, rounded to
// nearest, in forms that issue fewer instructions on the GPU than the plain
// operators while returning the same bits.
//
// The GPU has no single correctly rounded binary64 divide or square root;
// the compiler expands `n / d` into: scale d and n away from the extremes of
// the exponent range (v_div_scale), refine a reciprocal estimate of the
// scaled d by two Newton-Raphson steps, form the quotient, correct it with
// one fused remainder step (Markstein), undo the scaling (v_div_fmas) and
// patch zeros, infinities and NaNs (v_div_fixup).  The reciprocal part
// depends only on the scaled divisor, so two quotients by the same divisor
// can share it whenever the divisor scales the same way for both
// numerators -- checked lane by lane, so the sequence each lane runs is
// exactly the compiler's.
//
// `sqrt(x)` expands into a reciprocal square root estimate refined by
// Goldschmidt's coupled iteration (g ~ sqrt(x), h ~ 1/(2 sqrt(x))) with two
// fused correction steps, wrapped in a rescaling of arguments below 2^-767
// and a patch for 0 and +inf.  For arguments in [2^-767, +inf) those
// wrappers are identities; when every active lane of the wave has such an
// argument the wave runs the core alone, otherwise it calls sqrt().
//
// On the host every function is the plain operator.
#pragma once

#include <math.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sw {

// max(0, min(q, 1)), NaN and -0 to +0 (the minmod-type limiter of the Euler
// scheme): one maximum with the clamp output modifier on the GPU.
__host__ __device__ __forceinline__ double limiter(double q)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_fmin(__builtin_fmax(q, 0.0), 1.0);
#else
    if (q > 0.0)
        return q < 1.0 ? q : 1.0;
    return 0.0;
#endif
}

// A divisor with its scaled value and refined reciprocal (GPU), for
// several quotients by the same divisor.
struct RnDiv {
    double d;
    double ds;  // d scaled for the first numerator
    double r;   // refined reciprocal of ds
};

#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ double rn_recip(double ds)
{
    double r = __builtin_amdgcn_rcp(ds);
    double e = __builtin_fma(-ds, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-ds, r, 1.0);
    return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double rn_quotient(double n, double d, double ds, double r)
{
    bool scaled;
    const double ns = __builtin_amdgcn_div_scale(n, d, true, &scaled);
    const double q = ns * r;
    const double rem = __builtin_fma(-ds, q, ns);
    return __builtin_amdgcn_div_fixup(__builtin_amdgcn_div_fmas(rem, r, q, scaled), d, n);
}
#endif

// n / d, keeping what a second quotient by d can reuse in `dv`
__host__ __device__ __forceinline__ double rn_div_keep(double n, double d, RnDiv &dv)
{
    dv.d = d;
#if defined(__HIP_DEVICE_COMPILE__)
    bool unused;
    dv.ds = __builtin_amdgcn_div_scale(n, d, false, &unused);
    dv.r = rn_recip(dv.ds);
    return rn_quotient(n, d, dv.ds, dv.r);
#else
    dv.ds = d;
    dv.r = 0.0;
    return n / d;
#endif
}

// n / dv.d: reuses dv's reciprocal on the lanes where d scales as it did for
// the first numerator, and refines a new one on the others
__host__ __device__ __forceinline__ double rn_div_again(double n, const RnDiv &dv)
{
#if defined(__HIP_DEVICE_COMPILE__)
    bool unused;
    const double ds = __builtin_amdgcn_div_scale(n, dv.d, false, &unused);
    double r = dv.r;
    if (__double_as_longlong(ds) != __double_as_longlong(dv.ds)) {
        // an empty statement with side effects keeps this a branch the wave
        // skips, rather than a refinement run on every lane and discarded
        asm volatile("");
        r = rn_recip(ds);
    }
    return rn_quotient(n, dv.d, ds, r);
#else
    return n / dv.d;
#endif
}

#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ double rn_sqrt_core(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = y * 0.5;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double e = __builtin_fma(-g, g, x);
    g = __builtin_fma(e, h, g);
    e = __builtin_fma(-g, g, x);
    return __builtin_fma(e, h, g);
}

// x in [2^-767, +inf): the high word lies in [0x10000000, 0x7ff00000)
__device__ __forceinline__ uint32_t rn_sqrt_offset(double x)
{
    return (uint32_t)(__double2hiint(x)) - 0x10000000u;
}
#endif

// sqrt(x) and sqrt(y), rounded to nearest
__host__ __device__ __forceinline__ void rn_sqrt2(double x, double y, double &sx, double &sy)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t ox = rn_sqrt_offset(x), oy = rn_sqrt_offset(y);
    const uint32_t o = ox > oy ? ox : oy;
    if (__all(o < 0x7ff00000u - 0x10000000u)) {
        sx = rn_sqrt_core(x);
        sy = rn_sqrt_core(y);
    } else {
        sx = sqrt(x);
        sy = sqrt(y);
    }
#else
    sx = sqrt(x);
    sy = sqrt(y);
#endif
}

} // namespace sw
