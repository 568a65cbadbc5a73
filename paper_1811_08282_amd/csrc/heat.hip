// heat.hip -- heat-equation kernels (FTCS, Sec. 4.2): swept phases and the
// classic per-step kernel, binary64 and binary32 + Kahan.
//
// Cell update (difference form, evaluated exactly as written):
//     u' = u + r * ((u_right - u) + (u_left - u))
// binary32 adds Kahan compensation c to the increment:
//     d = r * (...);  y = d - c;  t = u + y;  c' = (t - u) - y;  u' = t
//
// Swept phase kernel: one workgroup per tile of W cells.  The tile and its
// two halo cells are staged in LDS as the two-slot working struct (slot
// m & 1 holds level m, Sec. 4.1: "at least two values ... alternate reading
// and writing"), the phase's window of levels is swept in LDS, and the W
// owned cells are written back.  Tiles of one phase write disjoint cells and
// read their halos from the previous phase's array, so phases ping-pong
// between two working arrays and no tile ever reads a cell another tile of
// the same launch writes.
#include "geom.h"
#include "kernels.h"

namespace sw {
namespace {

constexpr int kNaiveBlock = 256;

__device__ __forceinline__ int64_t wrap_cell(int64_t g, int64_t n)
{
    if (g < 0)
        return g + n;
    if (g >= n)
        return g - n;
    return g;
}

__device__ __forceinline__ double heat_update(double l, double c, double r_, double r)
{
    return c + r * ((r_ - c) + (l - c));
}

__global__ void __launch_bounds__(256)
k_heat_f64_phase(double *__restrict__ state, const double *__restrict__ ws_in,
                 double *__restrict__ ws_out, int64_t n, int w, int64_t offset, int64_t base,
                 int j_first, int j_last, double r, int first, int last)
{
    extern __shared__ double lds[];
    const int wp = w + 2;
    double *s0 = lds;
    double *s1 = lds + wp;
    // global cell of LDS index 0 (the left halo)
    const int64_t g0 = offset + (int64_t)blockIdx.x * w - 1;

    for (int i = threadIdx.x; i < wp; i += blockDim.x) {
        const int64_t g = wrap_cell(g0 + i, n);
        if (first) {
            s0[i] = state[g];
        } else {
            s0[i] = ws_in[g];
            s1[i] = ws_in[n + g];
        }
    }
    __syncthreads();

    for (int j = j_first; j <= j_last; ++j) {
        const int a = window_margin(j);
        const int64_t m = base + j;
        const double *src = (m & 1) ? s0 : s1;
        double *dst = (m & 1) ? s1 : s0;
        for (int i = a + 1 + threadIdx.x; i <= w - a; i += blockDim.x)
            dst[i] = heat_update(src[i - 1], src[i], src[i + 1], r);
        __syncthreads();
    }

    const bool top_odd = ((base + j_last) & 1) != 0;
    for (int i = 1 + threadIdx.x; i <= w; i += blockDim.x) {
        const int64_t g = wrap_cell(g0 + i, n);
        if (last) {
            state[g] = top_odd ? s1[i] : s0[i];
        } else {
            ws_out[g] = s0[i];
            ws_out[n + g] = s1[i];
        }
    }
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

// ---- binary32 + Kahan ----------------------------------------------------

__device__ __forceinline__ float heat_update_kahan(float l, float c, float rr, float r, float &comp)
{
    const float d = r * ((rr - c) + (l - c));
    const float y = d - comp;
    const float t = c + y;
    comp = (t - c) - y;
    return t;
}

__global__ void __launch_bounds__(256)
k_heat_f32_phase(float *__restrict__ state, const float *__restrict__ ws_in,
                 float *__restrict__ ws_out, int64_t n, int w, int64_t offset, int64_t base,
                 int j_first, int j_last, float r, int first, int last)
{
    extern __shared__ float ldsf[];
    const int wp = w + 2;
    float *s0 = ldsf;
    float *s1 = ldsf + wp;
    float *cc = ldsf + 2 * wp;
    const int64_t g0 = offset + (int64_t)blockIdx.x * w - 1;

    for (int i = threadIdx.x; i < wp; i += blockDim.x) {
        const int64_t g = wrap_cell(g0 + i, n);
        if (first) {
            s0[i] = state[g];
            cc[i] = state[n + g];
        } else {
            s0[i] = ws_in[g];
            s1[i] = ws_in[n + g];
            cc[i] = ws_in[2 * n + g];
        }
    }
    __syncthreads();

    for (int j = j_first; j <= j_last; ++j) {
        const int a = window_margin(j);
        const int64_t m = base + j;
        const float *src = (m & 1) ? s0 : s1;
        float *dst = (m & 1) ? s1 : s0;
        for (int i = a + 1 + threadIdx.x; i <= w - a; i += blockDim.x) {
            float comp = cc[i];
            dst[i] = heat_update_kahan(src[i - 1], src[i], src[i + 1], r, comp);
            cc[i] = comp;
        }
        __syncthreads();
    }

    const bool top_odd = ((base + j_last) & 1) != 0;
    for (int i = 1 + threadIdx.x; i <= w; i += blockDim.x) {
        const int64_t g = wrap_cell(g0 + i, n);
        if (last) {
            state[g] = top_odd ? s1[i] : s0[i];
            state[n + g] = cc[i];
        } else {
            ws_out[g] = s0[i];
            ws_out[n + g] = s1[i];
            ws_out[2 * n + g] = cc[i];
        }
    }
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

int phase_threads(int w)
{
    int t = ((w + 63) / 64) * 64;
    return t < 64 ? 64 : (t > 256 ? 256 : t);
}

} // namespace

hipError_t heat_f64_swept_phase(const PhaseLaunch &p, double *state, const double *ws_in,
                                double *ws_out, double r, hipStream_t s)
{
    const int64_t tiles = p.n / p.w;
    const size_t lds = (size_t)(p.w + 2) * kLdsPerCellHeatF64;
    hipLaunchKernelGGL(k_heat_f64_phase, dim3((unsigned)tiles), dim3(phase_threads(p.w)), lds, s,
                       state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, r,
                       (int)p.first, (int)p.last);
    return hipGetLastError();
}

hipError_t heat_f64_naive_step(const double *u, double *v, int64_t n, double r, hipStream_t s)
{
    const int64_t blocks = (n + kNaiveBlock - 1) / kNaiveBlock;
    hipLaunchKernelGGL(k_heat_f64_naive, dim3((unsigned)blocks), dim3(kNaiveBlock), 0, s, u, v, n,
                       r);
    return hipGetLastError();
}

hipError_t heat_f32_swept_phase(const PhaseLaunch &p, float *state, const float *ws_in,
                                float *ws_out, float r, hipStream_t s)
{
    const int64_t tiles = p.n / p.w;
    const size_t lds = (size_t)(p.w + 2) * kLdsPerCellHeatF32;
    hipLaunchKernelGGL(k_heat_f32_phase, dim3((unsigned)tiles), dim3(phase_threads(p.w)), lds, s,
                       state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, r,
                       (int)p.first, (int)p.last);
    return hipGetLastError();
}

hipError_t heat_f32_naive_step(const float *u, float *v, float *c, int64_t n, float r,
                               hipStream_t s)
{
    const int64_t blocks = (n + kNaiveBlock - 1) / kNaiveBlock;
    hipLaunchKernelGGL(k_heat_f32_naive, dim3((unsigned)blocks), dim3(kNaiveBlock), 0, s, u, v, c,
                       n, r);
    return hipGetLastError();
}

} // namespace sw
