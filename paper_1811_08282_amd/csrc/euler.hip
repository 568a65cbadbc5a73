// euler.hip -- 1D Euler kernels: the swept phase kernel (one workgroup per
// tile, body in tile_euler.h) and the classic sub-step kernels, binary64 and
// binary32 (+ Kahan, binary64 islands).  The classic kernels share each face
// flux (and each pressure) between the two cells of a block that use it.
#include "kernels.h"
#include "tile_euler.h"

namespace sw {
namespace {

constexpr int kNaiveBlock = 256;

template <int NT, int WT>
__global__ void __launch_bounds__(NT)
k_euler_f64_phase(double *__restrict__ state, const double *__restrict__ ws_in,
                  double *__restrict__ ws_out, int64_t n, int w, int64_t offset, int64_t base,
                  int j_first, int j_last, double lam, int first, int last)
{
    extern __shared__ double lds[];
    TileJob jb{state, ws_in, ws_out, n, offset + (int64_t)blockIdx.x * w - 1, base, lam, w,
               j_first, j_last, first, last, base + j_last};
    euler_f64_tile<NT, WT>(jb, lds);
}

template <int NT, int WT>
__global__ void __launch_bounds__(NT)
k_euler_f32_phase(float *__restrict__ state, const void *__restrict__ ws_in,
                  void *__restrict__ ws_out, int64_t n, int w, int64_t offset, int64_t base,
                  int j_first, int j_last, float lam, int first, int last)
{
    extern __shared__ double ldsd[];
    TileJob jb{state, ws_in, ws_out, n, offset + (int64_t)blockIdx.x * w - 1, base, (double)lam,
               w, j_first, j_last, first, last, base + j_last};
    euler_f32_tile<NT, WT>(jb, ldsd);
}

// Classic pressure-ratio sub-step: q (3n) -> pr (n).  Block-local pressures.
__global__ void __launch_bounds__(kNaiveBlock)
k_euler_f64_naive_pr(const double *__restrict__ q, double *__restrict__ pr, int64_t n)
{
    __shared__ double p[kNaiveBlock + 2];
    const int64_t b0 = (int64_t)blockIdx.x * kNaiveBlock;
    const int nloc = (int)((n - b0) < kNaiveBlock ? (n - b0) : kNaiveBlock);
    for (int i = threadIdx.x; i < nloc + 2; i += blockDim.x) {
        const int64_t g = wrap_cell(b0 - 1 + i, n);
        p[i] = pressure64(q[g], q[n + g], q[2 * n + g]);
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i < nloc)
        pr[b0 + i] = ratio(p[i], p[i + 1], p[i + 2]);
}

// Classic flux sub-step: predictor (t = 1: q1 = q0 + lam/2 dF(q0)) or
// corrector (t = 3: q0 += lam dF(q1)).  Block-local face fluxes.
__global__ void __launch_bounds__(kNaiveBlock)
k_euler_f64_naive_flux(int t, double *__restrict__ q0, double *__restrict__ q1,
                       const double *__restrict__ pr, int64_t n, double lam)
{
    __shared__ double f[3][kNaiveBlock + 1];
    const int64_t b0 = (int64_t)blockIdx.x * kNaiveBlock;
    const int nloc = (int)((n - b0) < kNaiveBlock ? (n - b0) : kNaiveBlock);
    const double *q = (t == 1) ? q0 : q1;
    for (int i = threadIdx.x; i < nloc + 1; i += blockDim.x) {
        const int64_t gl = wrap_cell(b0 - 1 + i, n);
        const int64_t gr = wrap_cell(b0 + i, n);
        face64(q[gl], q[n + gl], q[2 * n + gl], q[gr], q[n + gr], q[2 * n + gr], pr[gl], pr[gr],
               f[0][i], f[1][i], f[2][i]);
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i >= nloc)
        return;
    const int64_t g = b0 + i;
    if (t == 1) {
        const double hl = 0.5 * lam;
        for (int k = 0; k < 3; ++k)
            q1[k * n + g] = q0[k * n + g] + hl * (f[k][i] - f[k][i + 1]);
    } else {
        for (int k = 0; k < 3; ++k)
            q0[k * n + g] = q0[k * n + g] + lam * (f[k][i] - f[k][i + 1]);
    }
}

__global__ void __launch_bounds__(kNaiveBlock)
k_euler_f32_naive_pr(const float *__restrict__ q, double *__restrict__ pr, int64_t n)
{
    __shared__ double p[kNaiveBlock + 2];
    const int64_t b0 = (int64_t)blockIdx.x * kNaiveBlock;
    const int nloc = (int)((n - b0) < kNaiveBlock ? (n - b0) : kNaiveBlock);
    for (int i = threadIdx.x; i < nloc + 2; i += blockDim.x) {
        const int64_t g = wrap_cell(b0 - 1 + i, n);
        p[i] = pressure32(q[g], q[n + g], q[2 * n + g]);
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i < nloc)
        pr[b0 + i] = ratio(p[i], p[i + 1], p[i + 2]);
}

// q0c: caller state (q0[3][n] then c[3][n])
__global__ void __launch_bounds__(kNaiveBlock)
k_euler_f32_naive_flux(int t, float *__restrict__ q0c, float *__restrict__ q1,
                       const double *__restrict__ pr, int64_t n, float lam)
{
    __shared__ float f[3][kNaiveBlock + 1];
    const int64_t b0 = (int64_t)blockIdx.x * kNaiveBlock;
    const int nloc = (int)((n - b0) < kNaiveBlock ? (n - b0) : kNaiveBlock);
    const float *q = (t == 1) ? q0c : q1;
    for (int i = threadIdx.x; i < nloc + 1; i += blockDim.x) {
        const int64_t gl = wrap_cell(b0 - 1 + i, n);
        const int64_t gr = wrap_cell(b0 + i, n);
        face32(q[gl], q[n + gl], q[2 * n + gl], q[gr], q[n + gr], q[2 * n + gr], pr[gl], pr[gr],
               f[0][i], f[1][i], f[2][i]);
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i >= nloc)
        return;
    const int64_t g = b0 + i;
    if (t == 1) {
        const float hl = 0.5f * lam;
        for (int k = 0; k < 3; ++k)
            q1[k * n + g] = q0c[k * n + g] + hl * (f[k][i] - f[k][i + 1]);
    } else {
        for (int k = 0; k < 3; ++k) {
            float c = q0c[(3 + k) * n + g];
            q0c[k * n + g] = kahan_add(q0c[k * n + g], lam * (f[k][i] - f[k][i + 1]), c);
            q0c[(3 + k) * n + g] = c;
        }
    }
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

hipError_t euler_f64_swept_phase(const PhaseLaunch &p, double *state, const double *ws_in,
                                 double *ws_out, double lam, hipStream_t s)
{
    const size_t lds = (size_t)(p.w + 2) * kLdsPerCellEulerF64;
    const dim3 g = dim3((unsigned)p.tiles);
    if (p.threads == 512) {
        switch (p.w) {  // the default launch of Euler tiles of 1024 cells and more
        case 1024: return launch_kernel(k_euler_f64_phase<512, 1024>, g, 512, lds, s,
            state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam,
            (int)p.first, (int)p.last);
        default: break;
        }
    }
    if (p.threads == 256) {
        switch (p.w) {  // widths with compile-time LDS offsets
        case 128: return launch_kernel(k_euler_f64_phase<256, 128>, g, 256, lds, s,
            state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam,
            (int)p.first, (int)p.last);
        case 256: return launch_kernel(k_euler_f64_phase<256, 256>, g, 256, lds, s,
            state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam,
            (int)p.first, (int)p.last);
        case 512: return launch_kernel(k_euler_f64_phase<256, 512>, g, 256, lds, s,
            state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam,
            (int)p.first, (int)p.last);
        case 1024: return launch_kernel(k_euler_f64_phase<256, 1024>, g, 256, lds, s,
            state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam,
            (int)p.first, (int)p.last);
        default: break;
        }
    }
    return launch_by_threads(p.threads, k_euler_f64_phase<64, 0>, k_euler_f64_phase<128, 0>, k_euler_f64_phase<256, 0>, k_euler_f64_phase<512, 0>, g, lds, s,
        state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam, (int)p.first,
        (int)p.last);
}

hipError_t euler_f64_naive_substep(int t, double *q0, double *q1, double *pr, int64_t n,
                                   double lam, hipStream_t s)
{
    const unsigned blocks = (unsigned)((n + kNaiveBlock - 1) / kNaiveBlock);
    if ((t & 1) == 0)
        hipLaunchKernelGGL(k_euler_f64_naive_pr, dim3(blocks), dim3(kNaiveBlock), 0, s,
                           t == 0 ? q0 : q1, pr, n);
    else
        hipLaunchKernelGGL(k_euler_f64_naive_flux, dim3(blocks), dim3(kNaiveBlock), 0, s, t, q0, q1,
                           pr, n, lam);
    return hipGetLastError();
}

hipError_t euler_f32_swept_phase(const PhaseLaunch &p, float *state, const void *ws_in,
                                 void *ws_out, float lam, hipStream_t s)
{
    const size_t lds = (size_t)(p.w + 2) * kLdsPerCellEulerF32;
    const dim3 g = dim3((unsigned)p.tiles);
    if (p.threads == 512) {
        switch (p.w) {  // the default launch of Euler tiles of 1024 cells and more
        case 1024: return launch_kernel(k_euler_f32_phase<512, 1024>, g, 512, lds, s,
            state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam,
            (int)p.first, (int)p.last);
        default: break;
        }
    }
    if (p.threads == 256) {
        switch (p.w) {  // widths with compile-time LDS offsets
        case 256: return launch_kernel(k_euler_f32_phase<256, 256>, g, 256, lds, s,
            state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam,
            (int)p.first, (int)p.last);
        case 512: return launch_kernel(k_euler_f32_phase<256, 512>, g, 256, lds, s,
            state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam,
            (int)p.first, (int)p.last);
        case 1024: return launch_kernel(k_euler_f32_phase<256, 1024>, g, 256, lds, s,
            state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam,
            (int)p.first, (int)p.last);
        default: break;
        }
    }
    return launch_by_threads(p.threads, k_euler_f32_phase<64, 0>, k_euler_f32_phase<128, 0>, k_euler_f32_phase<256, 0>, k_euler_f32_phase<512, 0>, g, lds, s,
        state, ws_in, ws_out, p.n, p.w, p.offset, p.base, p.j_first, p.j_last, lam, (int)p.first,
        (int)p.last);
}

hipError_t euler_f32_naive_substep(int t, float *q0c, float *q1, double *pr, int64_t n, float lam,
                                   hipStream_t s)
{
    const unsigned blocks = (unsigned)((n + kNaiveBlock - 1) / kNaiveBlock);
    if ((t & 1) == 0)
        hipLaunchKernelGGL(k_euler_f32_naive_pr, dim3(blocks), dim3(kNaiveBlock), 0, s,
                           t == 0 ? q0c : q1, pr, n);
    else
        hipLaunchKernelGGL(k_euler_f32_naive_flux, dim3(blocks), dim3(kNaiveBlock), 0, s, t, q0c,
                           q1, pr, n, lam);
    return hipGetLastError();
}

} // namespace sw
