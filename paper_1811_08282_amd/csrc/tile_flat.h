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
constexpr int kFlatLanes = 60;  // cells a wave updates per pass (lanes 2..61)

// One sub-step of a tile in one pass with one barrier: a wave covers 64
// consecutive cells, lane l holding cell x = (first cell) - 2 + l.  Every
// lane reads its cell's source state from LDS and computes its pressure;
// the ratio (lanes 1..62), the face on the left of the cell (lanes 2..62)
// and the face on the right (lanes 2..61) take their neighbours from the
// adjacent lanes by DPP shifts, so pressures, ratios and fluxes never pass
// through LDS.  Lanes 2..61 update their cells (60 per wave); the outer two
// lanes on each side only supply neighbours.
//
// LDS: q0[3][wp] q1[3][wp]   (doubles, wp = w + 4).  ws layout: Q0[3][n], Q1[3][n]
template <int NT, int WT = 0>
__device__ __forceinline__ void flat_f64_tile(const TileJob &jb, double *lds)
{
    const int w = WT > 0 ? WT : jb.w;  // compile-time width when WT > 0
    const int wp = w + 2 * kFlatRadius;
    constexpr int kWaves = NT / 64;
    const int64_t n = jb.n;
    double *q0 = lds;
    double *q1 = lds + 3 * wp;
    double *state = (double *)jb.state;
    const double *ws_in = (const double *)jb.ws_in;
    double *ws_out = (double *)jb.ws_out;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid) >> 6;

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
    const bool updater = lane >= 2 && lane < 2 + kFlatLanes;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j, kFlatRadius);
        const int lo = a + kFlatRadius, hi = w - a + kFlatRadius;  // active LDS [lo, hi)
        const int t = (int)((jb.base + j - 1) & 1);
        const double *q = (t == 0) ? q0 : q1;
        const int chunks = (hi - lo + kFlatLanes - 1) / kFlatLanes;
        for (int k = wave; k < chunks; k += kWaves) {
            const int x = lo - 2 + kFlatLanes * k + lane;
            const int xc = x < hi + 1 ? x : hi + 1;  // cells past hi + 1 feed no update
            const double r0 = q[xc], r1 = q[wp + xc], r2 = q[2 * wp + xc];
            const double p = pressure64(r0, r1, r2);
            const double rt = ratio(from_prev_lane(p), p, from_next_lane(p));
            double f0, f1, f2;
            face64(from_prev_lane(r0), from_prev_lane(r1), from_prev_lane(r2), r0, r1, r2,
                   from_prev_lane(rt), rt, f0, f1, f2);
            const double g0 = from_next_lane(f0);
            const double g1 = from_next_lane(f1);
            const double g2 = from_next_lane(f2);
            if (updater && x < hi) {
                if (t == 0) {  // predictor: Q1 from Q0 (this lane's own source values)
                    q1[x] = r0 + half_lam * (f0 - g0);
                    q1[wp + x] = r1 + half_lam * (f1 - g1);
                    q1[2 * wp + x] = r2 + half_lam * (f2 - g2);
                } else {       // corrector: Q0 += lambda * (fluxes of Q1)
                    q0[x] = q0[x] + lam * (f0 - g0);
                    q0[wp + x] = q0[wp + x] + lam * (f1 - g1);
                    q0[2 * wp + x] = q0[2 * wp + x] + lam * (f2 - g2);
                }
            }
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

// LDS: q0[3][wp], c[3][wp], q1[3][wp] (float)
// ws layout: q0[3][n], c[3][n], q1[3][n] floats
template <int NT, int WT = 0>
__device__ __forceinline__ void flat_f32_tile(const TileJob &jb, double *ldsd)
{
    const int w = WT > 0 ? WT : jb.w;  // compile-time width when WT > 0
    const int wp = w + 2 * kFlatRadius;
    constexpr int kWaves = NT / 64;
    const int64_t n = jb.n;
    float *fst = (float *)ldsd;  // q0[3], c[3], q1[3]
    float *q0 = fst;
    float *cc = fst + 3 * wp;
    float *q1 = fst + 6 * wp;
    float *state = (float *)jb.state;
    const float *win = (const float *)jb.ws_in;
    float *wout = (float *)jb.ws_out;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid) >> 6;

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
    const bool updater = lane >= 2 && lane < 2 + kFlatLanes;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j, kFlatRadius);
        const int lo = a + kFlatRadius, hi = w - a + kFlatRadius;
        const int t = (int)((jb.base + j - 1) & 1);
        const float *q = (t == 0) ? q0 : q1;
        const int chunks = (hi - lo + kFlatLanes - 1) / kFlatLanes;
        for (int k = wave; k < chunks; k += kWaves) {
            const int x = lo - 2 + kFlatLanes * k + lane;
            const int xc = x < hi + 1 ? x : hi + 1;
            const float r0 = q[xc], r1 = q[wp + xc], r2 = q[2 * wp + xc];
            const double p = pressure32(r0, r1, r2);
            const double rt = ratio(from_prev_lane(p), p, from_next_lane(p));
            float f0, f1, f2;
            face32(from_prev_lane(r0), from_prev_lane(r1), from_prev_lane(r2), r0, r1, r2,
                   from_prev_lane(rt), rt, f0, f1, f2);
            const float g0 = from_next_lane(f0);
            const float g1 = from_next_lane(f1);
            const float g2 = from_next_lane(f2);
            if (updater && x < hi) {
                if (t == 0) {
                    q1[x] = r0 + half_lam * (f0 - g0);
                    q1[wp + x] = r1 + half_lam * (f1 - g1);
                    q1[2 * wp + x] = r2 + half_lam * (f2 - g2);
                } else {
                    const float f[3] = {f0, f1, f2}, gg[3] = {g0, g1, g2};
                    for (int m = 0; m < 3; ++m) {
                        float comp = cc[m * wp + x];
                        q0[m * wp + x] = kahan_add(q0[m * wp + x], lam * (f[m] - gg[m]), comp);
                        cc[m * wp + x] = comp;
                    }
                }
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
