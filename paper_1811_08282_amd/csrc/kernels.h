// kernels.h -- internal launch interface between the host planner (api.cpp)
// and the HIP kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sw {

constexpr int kLdsBytes = 160 * 1024;  // LDS of one gfx950 compute unit

// Per-cell bytes of the swept working struct held in HBM (two copies of the
// working arrays are used, ping-ponged between phases).
constexpr int kStructBytesHeatF64 = 16;   // u at even / odd levels
constexpr int kStructBytesHeatF32 = 12;   // u even / odd, Kahan c
constexpr int kStructBytesEulerF64 = 56;  // Q0[3], Q1[3], Pr
constexpr int kStructBytesEulerF32 = 44;  // Q0[3], c[3], Q1[3] (f32), Pr (f64)
constexpr int kStructBytesFlatF64 = 48;   // Q0[3], Q1[3]
constexpr int kStructBytesFlatF32 = 36;   // Q0[3], c[3], Q1[3] (f32)
constexpr int kStructBytesKsF64 = 16;     // u at even / odd levels

// Cells of LDS padding beyond each halo of a heat tile: the ghost lanes of
// the register-blocked level sweep read (unused) values up to one lane of
// cells past the halo.
constexpr int kHeatLdsPad = 5;

// LDS bytes per tile cell of each swept kernel (struct + scratch).
constexpr int kLdsPerCellHeatF64 = 16;
constexpr int kLdsPerCellHeatF32 = 12;
constexpr int kLdsPerCellEulerF64 = 64;  // struct 56 + pressure 8
constexpr int kLdsPerCellEulerF32 = 52;  // struct 44 + pressure 8
constexpr int kLdsPerCellFlatF64 = 48;   // struct only: pressures, ratios, fluxes by lane shifts
constexpr int kLdsPerCellFlatF32 = 36;   // struct only
constexpr int kLdsPerCellKsF64 = 16;     // struct only

// LDS cells of one tile of width w with stencil radius `radius`: the tile, its
// halos and, for heat, the padding.
inline int lds_tile_cells(bool heat, int w, int radius)
{
    return w + 2 * radius + (heat ? 2 * kHeatLdsPad : 0);
}

// Description of one swept phase launch.
struct PhaseLaunch {
    int64_t n;        // cells
    int w;            // tile width
    int64_t offset;   // first cell of the launch's first tile (the tiling's offset, 0 or
                      // w/2, plus w times the index of that tile)
    int64_t tiles;    // tiles (workgroups) of the launch: n / w, or the GPU's share
    int64_t base;     // (k - 1) * w/2
    int j_first, j_last;
    bool first;       // reads the caller's state (level 0 of this call)
    bool last;        // writes the caller's state (final level)
    int threads;      // workgroup size: 64, 128, 256 or 512
};

// Workgroup size of a swept phase for tile width w: whole waves covering the
// tile, at most 256 (the host raises Euler tiles of 1000 cells and more to 512).
inline int default_phase_threads(int w)
{
    const int t = ((w + 63) / 64) * 64;
    return t < 64 ? 64 : (t > 256 ? 256 : t);
}

// Heat, binary64.  state: u[n]; ws_in / ws_out: working arrays of 2n doubles.
hipError_t heat_f64_swept_phase(const PhaseLaunch &p, double *state, const double *ws_in,
                                double *ws_out, double r, hipStream_t s);
hipError_t heat_f64_naive_step(const double *u, double *v, int64_t n, double r, hipStream_t s);

// Heat, binary32 + Kahan.  state: u[n], c[n]; ws: 3n floats (u even, u odd, c).
hipError_t heat_f32_swept_phase(const PhaseLaunch &p, float *state, const float *ws_in,
                                float *ws_out, float r, hipStream_t s);
hipError_t heat_f32_naive_step(const float *u, float *v, float *c, int64_t n, float r,
                               hipStream_t s);

// Euler, binary64.  state: rho, m, E [n each]; ws: 7n doubles (Q0[3], Q1[3], Pr).
hipError_t euler_f64_swept_phase(const PhaseLaunch &p, double *state, const double *ws_in,
                                 double *ws_out, double lam, hipStream_t s);
// One classic sub-step of type t = 0..3 (Pr(Q0), predictor, Pr(Q1), corrector).
// q0: caller state (3n), q1: predictor state (3n), pr: pressure ratio (n).
hipError_t euler_f64_naive_substep(int t, double *q0, double *q1, double *pr, int64_t n,
                                   double lam, hipStream_t s);

// Euler, binary32 + Kahan + binary64 islands.  state: rho, m, E, c_rho, c_m,
// c_E [n floats each]; ws: 9n floats (Q0[3], c[3], Q1[3]) + n doubles (Pr).
hipError_t euler_f32_swept_phase(const PhaseLaunch &p, float *state, const void *ws_in,
                                 void *ws_out, float lam, hipStream_t s);
hipError_t euler_f32_naive_substep(int t, float *q0c, float *q1, double *pr, int64_t n,
                                   float lam, hipStream_t s);

// Euler, flattened layout (two five-point sub-steps per step), binary64:
// ws: Q0[3][n], Q1[3][n]; classic sub-step t = 0 predictor, 1 corrector.
hipError_t flat_f64_swept_phase(const PhaseLaunch &p, double *state, const double *ws_in,
                                double *ws_out, double lam, hipStream_t s);
hipError_t flat_f64_naive_substep(int t, double *q0, double *q1, int64_t n, double lam,
                                  hipStream_t s);
// binary32: ws: q0[3][n], c[3][n], q1[3][n] floats; classic q0c = caller state.
hipError_t flat_f32_swept_phase(const PhaseLaunch &p, float *state, const float *ws_in,
                                float *ws_out, float lam, hipStream_t s);
hipError_t flat_f32_naive_substep(int t, float *q0c, float *q1, int64_t n, float lam,
                                  hipStream_t s);

// Kuramoto-Sivashinsky, binary64.  state: u[n]; ws: slot0[n], slot1[n];
// a = dt / (2 dx), b = dt / dx^2, c = dt / dx^4.
hipError_t ks_f64_swept_phase(const PhaseLaunch &p, double *state, const double *ws_in,
                              double *ws_out, double a, double b, double c, hipStream_t s);
hipError_t ks_f64_naive_step(const double *u, double *v, int64_t n, double a, double b, double c,
                             hipStream_t s);

} // namespace sw
