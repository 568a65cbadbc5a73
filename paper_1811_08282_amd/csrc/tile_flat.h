// tile_flat.h -- one swept tile-phase of the "flattened" Euler layout
// (Sec. 4.3, Fig. 2a): two sub-steps per time step, each a five-point
// stencil that recomputes the pressure ratio on the fly, on a struct of six
// values per cell (Q0 and Q1; the paper's flattened version carries six
// doubles per point because the ratio is rolled into the step).
//
//   sub-step 0 (predictor)  Q1_i = Q0_i + (lambda/2)(F_{i-1/2}(Q0) - F_{i+1/2}(Q0))
//   sub-step 1 (corrector)  Q0_i = Q0_i + lambda (F_{i-1/2}(Q1) - F_{i+1/2}(Q1))
//
// with the same pressure ratio, limiter and Rusanov flux as the lengthened
// layout (tile_euler.h), evaluated in the same order, so both layouts give
// bit-identical states after every time step.  Radius 2 doubles every
// margin of the swept geometry (geom.h): H = W/4 levels per half phase, two
// halo cells per side.  A neighbour within two cells is at most one level
// ahead and then has overwritten only the field the cell no longer reads
// (Q1 after a predictor, Q0 after a corrector), so one struct suffices.
#pragma once

#include "geom.h"
#include "tile_euler.h"
#include "tile_job.h"

namespace sw {

constexpr int kFlatRadius = 2;

// LDS: q0[3][wp] q1[3][wp] P[wp] R[wp] tmp[3][wp]   (doubles, wp = w + 4)
// ws layout: Q0[3][n], Q1[3][n]
template <int NT, int WT = 0>
__device__ __forceinline__ void flat_f64_tile(const TileJob &jb, double *lds)
{
    const int w = WT > 0 ? WT : jb.w;  // compile-time width when WT > 0
    const int wp = w + 2 * kFlatRadius;
    const int64_t n = jb.n;
    double *q0 = lds;
    double *q1 = lds + 3 * wp;
    double *pp = lds + 6 * wp;
    double *pr = lds + 7 * wp;
    double *tmp = lds + 8 * wp;
    double *state = (double *)jb.state;
    const double *ws_in = (const double *)jb.ws_in;
    double *ws_out = (double *)jb.ws_out;
    const int tid = threadIdx.x;

    for (int i = tid; i < wp; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.first) {
            for (int k = 0; k < 3; ++k)
                q0[k * wp + i] = state[k * n + g];
        } else {
            for (int k = 0; k < 6; ++k)
                lds[k * wp + i] = ws_in[k * n + g];
        }
    }
    __syncthreads();

    const double lam = jb.coef;
    const double half_lam = 0.5 * lam;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j, kFlatRadius);
        const int lo = a + kFlatRadius, hi = w - a + kFlatRadius;  // active LDS [lo, hi)
        const int t = (int)((jb.base + j - 1) & 1);
        const double *q = (t == 0) ? q0 : q1;
        for (int i = lo - 2 + tid; i < hi + 2; i += NT)
            pp[i] = pressure64(q[i], q[wp + i], q[2 * wp + i]);
        __syncthreads();
        for (int i = lo - 1 + tid; i < hi + 1; i += NT)
            pr[i] = ratio(pp[i - 1], pp[i], pp[i + 1]);
        __syncthreads();
        for (int i = lo + tid; i < hi + 1; i += NT)
            face64(q[i - 1], q[wp + i - 1], q[2 * wp + i - 1], q[i], q[wp + i], q[2 * wp + i],
                   pr[i - 1], pr[i], tmp[i], tmp[wp + i], tmp[2 * wp + i]);
        __syncthreads();
        if (t == 0) {
            for (int i = lo + tid; i < hi; i += NT)
                for (int k = 0; k < 3; ++k)
                    q1[k * wp + i] =
                        q0[k * wp + i] + half_lam * (tmp[k * wp + i] - tmp[k * wp + i + 1]);
        } else {
            for (int i = lo + tid; i < hi; i += NT)
                for (int k = 0; k < 3; ++k)
                    q0[k * wp + i] = q0[k * wp + i] + lam * (tmp[k * wp + i] - tmp[k * wp + i + 1]);
        }
        __syncthreads();
    }

    for (int i = kFlatRadius + tid; i < w + kFlatRadius; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            for (int k = 0; k < 3; ++k)
                state[k * n + g] = q0[k * wp + i];
        } else {
            for (int k = 0; k < 6; ++k)
                ws_out[k * n + g] = lds[k * wp + i];
        }
    }
}

// LDS: P[wp], R[wp] (double), tmp[3][wp], q0[3][wp], c[3][wp], q1[3][wp] (float)
// ws layout: q0[3][n], c[3][n], q1[3][n] floats
template <int NT, int WT = 0>
__device__ __forceinline__ void flat_f32_tile(const TileJob &jb, double *ldsd)
{
    const int w = WT > 0 ? WT : jb.w;  // compile-time width when WT > 0
    const int wp = w + 2 * kFlatRadius;
    const int64_t n = jb.n;
    double *pp = ldsd;
    double *pr = ldsd + wp;
    float *ftmp = (float *)(ldsd + 2 * wp);
    float *fst = ftmp + 3 * wp;  // q0[3], c[3], q1[3]
    float *q0 = fst;
    float *cc = fst + 3 * wp;
    float *q1 = fst + 6 * wp;
    float *state = (float *)jb.state;
    const float *win = (const float *)jb.ws_in;
    float *wout = (float *)jb.ws_out;
    const int tid = threadIdx.x;

    for (int i = tid; i < wp; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.first) {
            for (int k = 0; k < 6; ++k)
                fst[k * wp + i] = state[k * n + g];
        } else {
            for (int k = 0; k < 9; ++k)
                fst[k * wp + i] = win[k * n + g];
        }
    }
    __syncthreads();

    const float lam = (float)jb.coef;
    const float half_lam = 0.5f * lam;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j, kFlatRadius);
        const int lo = a + kFlatRadius, hi = w - a + kFlatRadius;
        const int t = (int)((jb.base + j - 1) & 1);
        const float *q = (t == 0) ? q0 : q1;
        for (int i = lo - 2 + tid; i < hi + 2; i += NT)
            pp[i] = pressure32(q[i], q[wp + i], q[2 * wp + i]);
        __syncthreads();
        for (int i = lo - 1 + tid; i < hi + 1; i += NT)
            pr[i] = ratio(pp[i - 1], pp[i], pp[i + 1]);
        __syncthreads();
        for (int i = lo + tid; i < hi + 1; i += NT)
            face32(q[i - 1], q[wp + i - 1], q[2 * wp + i - 1], q[i], q[wp + i], q[2 * wp + i],
                   pr[i - 1], pr[i], ftmp[i], ftmp[wp + i], ftmp[2 * wp + i]);
        __syncthreads();
        if (t == 0) {
            for (int i = lo + tid; i < hi; i += NT)
                for (int k = 0; k < 3; ++k)
                    q1[k * wp + i] =
                        q0[k * wp + i] + half_lam * (ftmp[k * wp + i] - ftmp[k * wp + i + 1]);
        } else {
            for (int i = lo + tid; i < hi; i += NT)
                for (int k = 0; k < 3; ++k) {
                    float c = cc[k * wp + i];
                    q0[k * wp + i] = kahan_add(q0[k * wp + i],
                                               lam * (ftmp[k * wp + i] - ftmp[k * wp + i + 1]), c);
                    cc[k * wp + i] = c;
                }
        }
        __syncthreads();
    }

    for (int i = kFlatRadius + tid; i < w + kFlatRadius; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            for (int k = 0; k < 6; ++k)
                state[k * n + g] = fst[k * wp + i];
        } else {
            for (int k = 0; k < 9; ++k)
                wout[k * n + g] = fst[k * wp + i];
        }
    }
}

} // namespace sw
