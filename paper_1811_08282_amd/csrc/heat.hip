// heat.hip -- heat-equation kernels (FTCS, Sec. 4.2): the swept phase kernel
// (one workgroup per tile, body in tile_heat.h) and the classic per-step
// kernel, binary64 and binary32 + Kahan.
#include "kernels.h"
#include "tile_heat.h"

namespace sw {
namespace {

constexpr int kNaiveBlock = 256;

template <int NT>
__global__ void __launch_bounds__(NT)
k_heat_f64_phase(double *__restrict__ state, const double *__restrict__ ws_in,
                 double *__restrict__ ws_out, int64_t n, int w, int64_t offset, int64_t base,
                 int j_first, int j_last, double r, int first, int last)
{
    extern __shared__ double lds[];
    TileJob jb{state, ws_in, ws_out, n, offset + (int64_t)blockIdx.x * w - 1, base, r, w,
               j_first, j_last, first, last};
    heat_f64_tile<NT>(jb, lds);
}

template <int NT>
__global__ void __launch_bounds__(NT)
k_heat_f32_phase(float *__restrict__ state, const float *__restrict__ ws_in,
                 float *__restrict__ ws_out, int64_t n, int w, int64_t offset, int64_t base,
                 int j_first, int j_last, float r, int first, int last)
{
    extern __shared__ float ldsf[];
    TileJob jb{state, ws_in, ws_out, n, offset + (int64_t)blockIdx.x * w - 1, base, (double)r, w,
               j_first, j_last, first, last};
    heat_f32_tile<NT>(jb, ldsf);
}

__global__ void __launch_bounds__(kNaiveBlock)
k_heat_f64_naive(const double *__restrict__ u, double *__restrict__ v, int64_t n, double r)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t il = (i == 0) ? n - 1 : i - 1;
    const int64_t ir = (i == n - 1) ? 0 : i + 1;
    v[i] = heat_update(u[il], u[i], u[ir], r);
}

__global__ void __launch_bounds__(kNaiveBlock)
k_heat_f32_naive(const float *__restrict__ u, float *__restrict__ v, float *__restrict__ c,
                 int64_t n, float r)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t il = (i == 0) ? n - 1 : i - 1;
    const int64_t ir = (i == n - 1) ? 0 : i + 1;
    float comp = c[i];
    v[i] = heat_update_kahan(u[il], u[i], u[ir], r, comp);
    c[i] = comp;
}

// Four consecutive cells per thread with 16-byte loads and stores (n a
// multiple of 4; arrays 16-byte aligned): the classic step at close to the
// memory rate.  Same update, same operation order as the one-cell kernel.
__global__ void __launch_bounds__(kNaiveBlock)
k_heat_f64_naive4(const double *__restrict__ u, double *__restrict__ v, int64_t n, double r)
{
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i0 >= n)
        return;
    const double2 a = *(const double2 *)(u + i0);
    const double2 b = *(const double2 *)(u + i0 + 2);
    const double l = u[i0 == 0 ? n - 1 : i0 - 1];
    const double rr = u[i0 + 4 == n ? 0 : i0 + 4];
    double2 o0, o1;
    o0.x = heat_update(l, a.x, a.y, r);
    o0.y = heat_update(a.x, a.y, b.x, r);
    o1.x = heat_update(a.y, b.x, b.y, r);
    o1.y = heat_update(b.x, b.y, rr, r);
    *(double2 *)(v + i0) = o0;
    *(double2 *)(v + i0 + 2) = o1;
}

__global__ void __launch_bounds__(kNaiveBlock)
k_heat_f32_naive4(const float *__restrict__ u, float *__restrict__ v, float *__restrict__ c,
                  int64_t n, float r)
{
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i0 >= n)
        return;
    const float4 a = *(const float4 *)(u + i0);
    float4 k = *(const float4 *)(c + i0);
    const float l = u[i0 == 0 ? n - 1 : i0 - 1];
    const float rr = u[i0 + 4 == n ? 0 : i0 + 4];
    float4 o;
    o.x = heat_update_kahan(l, a.x, a.y, r, k.x);
    o.y = heat_update_kahan(a.x, a.y, a.z, r, k.y);
    o.z = heat_update_kahan(a.y, a.z, a.w, r, k.z);
    o.w = heat_update_kahan(a.z, a.w, rr, r, k.w);
    *(float4 *)(v + i0) = o;
    *(float4 *)(c + i0) = k;
}

template <typename K64, typename K128, typename K256, typename K512, typename... Args>
hipError_t launch_by_threads(int nt, K64 k64, K128 k128, K256 k256, K512 k512, dim3 grid,
                             size_t lds, hipStream_t s, Args... args)
{
    if (nt == 64)
        hipLaunchKernelGGL(k64, grid, dim3(64), lds, s, args...);
    else if (nt == 128)
        hipLaunchKernelGGL(k128, grid, dim3(128), lds, s, args...);
    else if (nt == 256)
        hipLaunchKernelGGL(k256, grid, dim3(256), lds, s, args...);
    else
        hipLaunchKernelGGL(k512, grid, dim3(512), lds, s, args...);
    return hipGetLastError();
}

} // namespace

hipError_t heat_f64_swept_phase(const PhaseLaunch &p, double *state, const double *ws_in,
                                double *ws_out, double r, hipStream_t s)
{
    const size_t lds = (size_t)lds_tile_cells(true, p.w, 1) * kLdsPerCellHeatF64;
    return launch_by_threads(p.threads, k_heat_f64_phase<64>, k_heat_f64_phase<128>,
                             k_heat_f64_phase<256>, k_heat_f64_phase<512>, dim3((unsigned)p.tiles), lds, s, state,
                             ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, r,
                             (int)p.first, (int)p.last);
}

hipError_t heat_f64_naive_step(const double *u, double *v, int64_t n, double r, hipStream_t s)
{
    if ((n & 3) == 0) {
        const int64_t blocks = (n / 4 + kNaiveBlock - 1) / kNaiveBlock;
        hipLaunchKernelGGL(k_heat_f64_naive4, dim3((unsigned)blocks), dim3(kNaiveBlock), 0, s, u, v,
                           n, r);
        return hipGetLastError();
    }
    const int64_t blocks = (n + kNaiveBlock - 1) / kNaiveBlock;
    hipLaunchKernelGGL(k_heat_f64_naive, dim3((unsigned)blocks), dim3(kNaiveBlock), 0, s, u, v, n,
                       r);
    return hipGetLastError();
}

hipError_t heat_f32_swept_phase(const PhaseLaunch &p, float *state, const float *ws_in,
                                float *ws_out, float r, hipStream_t s)
{
    const size_t lds = (size_t)lds_tile_cells(true, p.w, 1) * kLdsPerCellHeatF32;
    return launch_by_threads(p.threads, k_heat_f32_phase<64>, k_heat_f32_phase<128>,
                             k_heat_f32_phase<256>, k_heat_f32_phase<512>, dim3((unsigned)p.tiles), lds, s, state,
                             ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, r,
                             (int)p.first, (int)p.last);
}

hipError_t heat_f32_naive_step(const float *u, float *v, float *c, int64_t n, float r,
                               hipStream_t s)
{
    if ((n & 3) == 0) {
        const int64_t blocks = (n / 4 + kNaiveBlock - 1) / kNaiveBlock;
        hipLaunchKernelGGL(k_heat_f32_naive4, dim3((unsigned)blocks), dim3(kNaiveBlock), 0, s, u, v,
                           c, n, r);
        return hipGetLastError();
    }
    const int64_t blocks = (n + kNaiveBlock - 1) / kNaiveBlock;
    hipLaunchKernelGGL(k_heat_f32_naive, dim3((unsigned)blocks), dim3(kNaiveBlock), 0, s, u, v, c,
                       n, r);
    return hipGetLastError();
}

} // namespace sw
