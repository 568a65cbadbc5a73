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
//
// Level sweep: each thread updates four consecutive cells.  It reads their
// eight-cell neighbourhood with four 16-byte LDS loads, forms the six second
// differences s_k and six fluxes f(u_k) between them once (instead of three
// and two per cell) and writes the four results with two 16-byte stores.
// Every window is a whole number of such groups and every group starts on an
// even cell: W is a multiple of 4 (the host's width rule for radius 2) and
// the margins 2|j - 1| are even, so the windows [m + 2, W - m + 2) of the
// LDS slots hold a multiple of 4 cells from an even index, and the slots
// (W + 4 doubles each) start on 32-byte boundaries.
#pragma once

#include "geom.h"
#include "tile_job.h"

namespace sw {

constexpr int kKsRadius = 2;
constexpr int kKsCells = 4;  // consecutive cells per thread and level
static_assert(kKsCells == 4, "the level sweep stores a group as two 16-byte halves");

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

// One level over the LDS window [lo, hi) (hi - lo a multiple of 4, lo even),
// from slot src to slot dst; reads [lo - 2, hi + 2).
template <int NT>
__device__ __forceinline__ void ks_level(const double *src, double *dst, int lo, int hi, double a,
                                         double b, double c)
{
    for (int x0 = lo + kKsCells * (int)threadIdx.x; x0 < hi; x0 += kKsCells * NT) {
        double u[kKsCells + 4], sd[kKsCells + 2], fl[kKsCells + 2], out[kKsCells];
        const double2 *in2 = reinterpret_cast<const double2 *>(src + x0 - 2);
#pragma unroll
        for (int k = 0; k < (kKsCells + 4) / 2; ++k) {  // cells x0 - 2 .. x0 + 5
            const double2 v = in2[k];
            u[2 * k] = v.x;
            u[2 * k + 1] = v.y;
        }
#pragma unroll
        for (int k = 0; k < kKsCells + 2; ++k) {  // cells x0 - 1 .. x0 + 4
            sd[k] = ks_second(u[k], u[k + 1], u[k + 2]);
            fl[k] = ks_flux(u[k + 1]);
        }
        // cell x0 + k: ks_update of u[k .. k + 4] with the shared terms
#pragma unroll
        for (int k = 0; k < kKsCells; ++k) {
            const double q = (sd[k + 2] - sd[k + 1]) + (sd[k] - sd[k + 1]);
            out[k] = u[k + 2] - ((a * (fl[k + 2] - fl[k]) + b * sd[k + 1]) + c * q);
        }
        double2 *out2 = reinterpret_cast<double2 *>(dst + x0);
        out2[0] = make_double2(out[0], out[1]);
        out2[1] = make_double2(out[2], out[3]);
    }
}

// LDS: s0[w+4], s1[w+4] doubles (LDS index = tile cell + 2).  ws layout:
// slot0[n], slot1[n].  One barrier per level.
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
        ks_level<NT>(src, dst, m + R, w - m + R, a, b, c);
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
