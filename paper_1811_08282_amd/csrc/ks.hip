// ks.hip -- Kuramoto-Sivashinsky kernels: the swept phase kernel (one
// workgroup per tile, body in tile_ks.h) and the classic per-step kernel,
// binary64.
#include "kernels.h"
#include "tile_ks.h"

namespace sw {
namespace {

constexpr int kNaiveBlock = 256;

template <int NT>
__global__ void __launch_bounds__(NT)
k_ks_f64_phase(double *__restrict__ state, const double *__restrict__ ws_in,
               double *__restrict__ ws_out, int64_t n, int w, int64_t offset, int64_t base,
               int j_first, int j_last, double a, double b, double c, int first, int last)
{
    extern __shared__ double lds[];
    TileJob jb{state, ws_in, ws_out, n, offset + (int64_t)blockIdx.x * w - kKsRadius, base, 0.0,
               w, j_first, j_last, first, last, base + j_last};
    ks_f64_tile<NT>(jb, lds, a, b, c);
}

// one time step from HBM: each work-item reads its five cells (neighbouring
// work-items share them through the caches) and writes one
__global__ void __launch_bounds__(kNaiveBlock)
k_ks_f64_naive(const double *__restrict__ u, double *__restrict__ v, int64_t n, double a,
               double b, double c)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t im = i == 0 ? n - 1 : i - 1;
    const int64_t imm = im == 0 ? n - 1 : im - 1;
    const int64_t ip = i == n - 1 ? 0 : i + 1;
    const int64_t ipp = ip == n - 1 ? 0 : ip + 1;
    v[i] = ks_update(u[imm], u[im], u[i], u[ip], u[ipp], a, b, c);
}

} // namespace

hipError_t ks_f64_swept_phase(const PhaseLaunch &p, double *state, const double *ws_in,
                              double *ws_out, double a, double b, double c, hipStream_t s)
{
    const size_t lds = (size_t)lds_tile_cells(false, p.w, kKsRadius) * kLdsPerCellKsF64;
    const dim3 g((unsigned)p.tiles);
    const int first = (int)p.first, last = (int)p.last;
    switch (p.threads) {
    case 64:
        hipLaunchKernelGGL(k_ks_f64_phase<64>, g, dim3(64), lds, s, state, ws_in, ws_out, p.n,
                           p.w, p.offset, p.base, p.j_first, p.j_last, a, b, c, first, last);
        break;
    case 128:
        hipLaunchKernelGGL(k_ks_f64_phase<128>, g, dim3(128), lds, s, state, ws_in, ws_out, p.n,
                           p.w, p.offset, p.base, p.j_first, p.j_last, a, b, c, first, last);
        break;
    case 256:
        hipLaunchKernelGGL(k_ks_f64_phase<256>, g, dim3(256), lds, s, state, ws_in, ws_out, p.n,
                           p.w, p.offset, p.base, p.j_first, p.j_last, a, b, c, first, last);
        break;
    default:
        hipLaunchKernelGGL(k_ks_f64_phase<512>, g, dim3(512), lds, s, state, ws_in, ws_out, p.n,
                           p.w, p.offset, p.base, p.j_first, p.j_last, a, b, c, first, last);
        break;
    }
    return hipGetLastError();
}

hipError_t ks_f64_naive_step(const double *u, double *v, int64_t n, double a, double b, double c,
                             hipStream_t s)
{
    const int64_t blocks = (n + kNaiveBlock - 1) / kNaiveBlock;
    hipLaunchKernelGGL(k_ks_f64_naive, dim3((unsigned)blocks), dim3(kNaiveBlock), 0, s, u, v, n, a,
                       b, c);
    return hipGetLastError();
}

} // namespace sw
