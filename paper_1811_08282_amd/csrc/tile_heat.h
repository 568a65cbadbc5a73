// tile_heat.h -- one swept tile-phase of the heat equation (FTCS, Sec. 4.2),
// as a device function run by a whole workgroup.  Used by the per-phase
// kernels and by the persistent batch kernel.
//
// Cell update (difference form, evaluated exactly as written):
//     u' = u + r * ((u_right - u) + (u_left - u))
// binary32 adds Kahan compensation c to the increment:
//     d = r * (...);  y = d - c;  t = u + y;  c' = (t - u) - y;  u' = t
//
// The tile and its two halo cells are staged in LDS as the two-slot working
// struct (slot m & 1 holds level m), the phase's window of levels is swept in
// LDS with one barrier per level, and the W owned cells are written back.
#pragma once

#include "geom.h"
#include "tile_job.h"

namespace sw {

__device__ __forceinline__ double heat_update(double l, double c, double r_, double r)
{
    return c + r * ((r_ - c) + (l - c));
}

__device__ __forceinline__ float heat_update_kahan(float l, float c, float rr, float r, float &comp)
{
    const float d = r * ((rr - c) + (l - c));
    const float y = d - comp;
    const float t = c + y;
    comp = (t - c) - y;
    return t;
}

// LDS: s0[w+2], s1[w+2] doubles.  ws layout: slot0[n], slot1[n].
template <int NT>
__device__ __forceinline__ void heat_f64_tile(const TileJob &jb, double *lds)
{
    const int w = jb.w;
    const int wp = w + 2;
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

    const double r = jb.coef;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j);
        const int64_t m = jb.base + j;
        const double *src = (m & 1) ? s0 : s1;
        double *dst = (m & 1) ? s1 : s0;
        for (int i = a + 1 + tid; i <= w - a; i += NT)
            dst[i] = heat_update(src[i - 1], src[i], src[i + 1], r);
        __syncthreads();
    }

    const bool top_odd = ((jb.base + jb.j_last) & 1) != 0;
    for (int i = 1 + tid; i <= w; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            state[g] = top_odd ? s1[i] : s0[i];
        } else {
            ws_out[g] = s0[i];
            ws_out[n + g] = s1[i];
        }
    }
}

// LDS: s0[w+2], s1[w+2], c[w+2] floats.  ws layout: u0[n], u1[n], c[n].
template <int NT>
__device__ __forceinline__ void heat_f32_tile(const TileJob &jb, float *ldsf)
{
    const int w = jb.w;
    const int wp = w + 2;
    const int64_t n = jb.n;
    float *s0 = ldsf;
    float *s1 = ldsf + wp;
    float *cc = ldsf + 2 * wp;
    float *state = (float *)jb.state;
    const float *ws_in = (const float *)jb.ws_in;
    float *ws_out = (float *)jb.ws_out;
    const int tid = threadIdx.x;

    for (int i = tid; i < wp; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.first) {
            s0[i] = state[g];
            cc[i] = state[n + g];
        } else {
            s0[i] = ws_in[g];
            s1[i] = ws_in[n + g];
            cc[i] = ws_in[2 * n + g];
        }
    }
    __syncthreads();

    const float r = (float)jb.coef;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j);
        const int64_t m = jb.base + j;
        const float *src = (m & 1) ? s0 : s1;
        float *dst = (m & 1) ? s1 : s0;
        // two cells per thread and pass (i and i + NT): the compiler pairs
        // their LDS accesses (three instructions per cell instead of five)
        // and shares the address arithmetic.  Measured 6 % faster at
        // W = 2048; the binary64 loop above is bound by LDS bandwidth, and
        // the same pairing there measured 13 % slower.
        const int end = w - a;
        int i = a + 1 + tid;
        for (; i + NT <= end; i += 2 * NT) {
            float c0 = cc[i], c1 = cc[i + NT];
            const float x0 = heat_update_kahan(src[i - 1], src[i], src[i + 1], r, c0);
            const float x1 = heat_update_kahan(src[i + NT - 1], src[i + NT], src[i + NT + 1], r, c1);
            dst[i] = x0;
            dst[i + NT] = x1;
            cc[i] = c0;
            cc[i + NT] = c1;
        }
        if (i <= end) {
            float comp = cc[i];
            dst[i] = heat_update_kahan(src[i - 1], src[i], src[i + 1], r, comp);
            cc[i] = comp;
        }
        __syncthreads();
    }

    const bool top_odd = ((jb.base + jb.j_last) & 1) != 0;
    for (int i = 1 + tid; i <= w; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            state[g] = top_odd ? s1[i] : s0[i];
            state[n + g] = cc[i];
        } else {
            ws_out[g] = s0[i];
            ws_out[n + g] = s1[i];
            ws_out[2 * n + g] = cc[i];
        }
    }
}

} // namespace sw
