// tile_ks.h -- the Kuramoto-Sivashinsky equation u_t + u u_x + u_xx + u_xxxx = 0
// (named in Sec. 2 among the equations the swept rule has been applied to)
// on the swept schedule: cell arithmetic (host and device) and one swept
// tile-phase as a device function run by a whole workgroup.
//
// Scheme: forward Euler in time, central differences; per cell, from the five
// cells u[i-2..i+2] of the previous level, evaluated exactly as written:
//   s_k = (u_{k+1} - u_k) + (u_{k-1} - u_k)            k = i-1, i, i+1
//   q   = (s_{i+1} - s_i) + (s_{i-1} - s_i)
//   u'  = u_i - ((a * (f(u_{i+1}) - f(u_{i-1})) + b * s_i) + c * q),  f(u) = 0.5 * (u * u)
// with a = dt / (2 dx), b = dt / dx^2, c = dt / dx^4.
//
// One sub-step per time step on a stencil of radius 2: the radius-2 swept
// geometry (margins 2|j - 1|, W/4 levels per half phase, two halo cells per
// side) with the two-slot working struct of the heat scheme (slot m & 1
// holds level m; a neighbour within two cells is at most one level ahead and
// writes only the slot the cell no longer reads).
#pragma once

#include "geom.h"
#include "tile_job.h"

namespace sw {

constexpr int kKsRadius = 2;

__host__ __device__ __forceinline__ double ks_second(double l, double m, double r)
{
    return (r - m) + (l - m);
}

__host__ __device__ __forceinline__ double ks_flux(double u)
{
    return 0.5 * (u * u);
}

__host__ __device__ __forceinline__ double ks_update(double umm, double um, double u, double up,
                                                     double upp, double a, double b, double c)
{
    const double sm = ks_second(umm, um, u);
    const double s0 = ks_second(um, u, up);
    const double sp = ks_second(u, up, upp);
    const double q = (sp - s0) + (sm - s0);
    return u - ((a * (ks_flux(up) - ks_flux(um)) + b * s0) + c * q);
}

// LDS: s0[w+4], s1[w+4] doubles (LDS index = tile cell + 2).  ws layout:
// slot0[n], slot1[n].  The level window is swept in LDS with one barrier per
// level.
template <int NT>
__device__ __forceinline__ void ks_f64_tile(const TileJob &jb, double *lds, double a, double b,
                                            double c)
{
    constexpr int R = kKsRadius;
    const int w = jb.w;
    const int wp = w + 2 * R;
    const int64_t n = jb.n;
    double *s0 = lds;
    double *s1 = lds + wp;
    double *state = (double *)jb.state;
    const double *ws_in = (const double *)jb.ws_in;
    double *ws_out = (double *)jb.ws_out;
    const int tid = threadIdx.x;

    for (int i = tid; i < wp; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.first) {
            s0[i] = state[g];
        } else {
            s0[i] = ws_in[g];
            s1[i] = ws_in[n + g];
        }
    }
    __syncthreads();

    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int m = window_margin(j, R);
        const int64_t lv = jb.base + j;
        const double *src = (lv & 1) ? s0 : s1;
        double *dst = (lv & 1) ? s1 : s0;
        for (int i = m + R + tid; i < w - m + R; i += NT)
            dst[i] = ks_update(src[i - 2], src[i - 1], src[i], src[i + 1], src[i + 2], a, b, c);
        __syncthreads();
    }

    const bool top_odd = ((jb.base + jb.j_last) & 1) != 0;
    for (int i = R + tid; i < w + R; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            state[g] = top_odd ? s1[i] : s0[i];
        } else {
            ws_out[g] = s0[i];
            ws_out[n + g] = s1[i];
        }
    }
}

} // namespace sw
