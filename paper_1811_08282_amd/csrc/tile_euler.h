// tile_euler.h -- Euler cell arithmetic and one swept tile-phase of the 1D
// Euler equations, as device functions.
//
// Scheme (Sec. 4.2: second-order finite volume with a minmod limiter; the
// lengthened layout of Sec. 4.3 / Fig. 2b: a per-cell struct of Q0, Q1 and
// the pressure ratio Pr, four three-point sub-steps per time step):
//   sub-step 0  Pr_i = (p_{i+1} - p_i) / (p_i - p_{i-1})      from Q0
//   sub-step 1  Q1_i = Q0_i + (lambda/2) (F_{i-1/2} - F_{i+1/2})  fluxes of Q0
//   sub-step 2  Pr_i                                          from Q1
//   sub-step 3  Q0_i = Q0_i + lambda (F_{i-1/2} - F_{i+1/2})     fluxes of Q1
// Face i+1/2 between cells L = i and R = i+1: limited states
//   U- = U_L + (phi(1/Pr_L)/2) (U_R - U_L),  U+ = U_R - (phi(Pr_R)/2) (U_R - U_L)
// with phi(q) = max(0, min(q, 1)) (NaN -> 0), and the Rusanov flux
//   F = (F(U-) + F(U+))/2 - (sigma/2) (U+ - U-),  sigma = max(|u-|+a-, |u+|+a+).
// gamma = 1.4, gamma - 1 = 0.4 as literals; every expression is evaluated in
// the written order (the library is built without contraction).
//
// A neighbour that is one level ahead never overwrites a field a cell still
// needs (Pr is written only at sub-steps 0/2, Q1 at 1, Q0 at 3), which is why
// one struct per cell carries both of its latest levels.
//
// Face sharing: inside a flux sub-step every face flux is computed once and
// used by both cells it separates, without going through LDS: each lane
// evaluates the face on the left of its cell and takes the face on the right
// from the next lane (a DPP lane shift), so a wave updates 63 cells and its
// last lane only evaluates the face the 63rd cell needs.  The sub-step then
// needs one barrier (after the update) instead of two.  Each cell's pressure
// is kept in LDS and refreshed whenever its state changes, so a ratio
// sub-step reads three stored pressures instead of recomputing them.
#pragma once

#include <math.h>

#include "geom.h"
#include "lanes.h"
#include "rn_ops.h"
#include "tile_job.h"

namespace sw {

constexpr double kGamma = 1.4;
constexpr double kGm1 = 0.4;

__host__ __device__ __forceinline__ double ratio(double pm, double pc, double pp)
{
    return (pp - pc) / (pc - pm);
}

constexpr int kFaceLanes = 63;  // cells a wave updates per pass (lane 63: face only)

// ---- binary64 ----------------------------------------------------------------

__host__ __device__ __forceinline__ double pressure64(double rho, double m, double e)
{
    const double u = m / rho;
    return kGm1 * (e - 0.5 * (m * u));
}

__host__ __device__ __forceinline__ void face64(double a0, double a1, double a2, double b0, double b1,
                                       double b2, double pra, double prb, double &f0, double &f1,
                                       double &f2)
{
    const double hl = 0.5 * limiter(1.0 / pra);
    const double hr = 0.5 * limiter(prb);
    const double d0 = b0 - a0, d1 = b1 - a1, d2 = b2 - a2;
    const double l0 = a0 + hl * d0, l1 = a1 + hl * d1, l2 = a2 + hl * d2;
    const double r0 = b0 - hr * d0, r1 = b1 - hr * d1, r2 = b2 - hr * d2;
    RnDiv dl, dr;  // l0 and r0 each divide twice
    const double vl = rn_div_keep(l1, l0, dl);
    const double pl = kGm1 * (l2 - 0.5 * (l1 * vl));
    const double vr = rn_div_keep(r1, r0, dr);
    const double pr = kGm1 * (r2 - 0.5 * (r1 * vr));
    double al, ar;
    rn_sqrt2(rn_div_again(kGamma * pl, dl), rn_div_again(kGamma * pr, dr), al, ar);
    const double sl = fabs(vl) + al;
    const double sr = fabs(vr) + ar;
    const double hs = 0.5 * (sl > sr ? sl : sr);
    f0 = 0.5 * (l1 + r1) - hs * (r0 - l0);
    f1 = 0.5 * ((l1 * vl + pl) + (r1 * vr + pr)) - hs * (r1 - l1);
    f2 = 0.5 * ((l2 + pl) * vl + (r2 + pr) * vr) - hs * (r2 - l2);
}

// top level of LDS cell i when a phase starts (halos: the previous peak)
__host__ __device__ __forceinline__ int64_t entry_level(const TileJob &jb, int i, int w)
{
    if (jb.first)
        return 0;
    const int64_t cap = jb.final_level;
    if (i == 0 || i == w + 1)
        return jb.base < cap ? jb.base : cap;
    const int o = i - 1;
    const int p = (o + 1 < w - o) ? o + 1 : w - o;
    int64_t lv = jb.base + 1 - p;
    lv = lv < 0 ? 0 : lv;
    return lv < cap ? lv : cap;
}

// LDS: q0[3][wp] q1[3][wp] pr[wp] P[wp]   (doubles, wp = w + 2)
// P holds the pressure of the state the next ratio sub-step reads: p(Q0) for
// a cell whose level is 0 or 1 mod 4, p(Q1) for 2 or 3 mod 4.  It is set
// from the entry level at load and refreshed by every predictor/corrector.
template <int NT, int WT = 0>
__device__ __forceinline__ void euler_f64_tile(const TileJob &jb, double *lds)
{
    const int w = WT > 0 ? WT : jb.w;  // compile-time width when WT > 0
    const int wp = w + 2;
    constexpr int kWaves = NT / 64;
    const int64_t n = jb.n;
    double *q0 = lds;
    double *q1 = lds + 3 * wp;
    double *pr = lds + 6 * wp;
    double *pp = lds + 7 * wp;
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
            pp[i] = pressure64(q0[i], q0[wp + i], q0[2 * wp + i]);
        } else {
            for (int k = 0; k < 7; ++k)
                lds[k * wp + i] = ws_in[k * n + g];
            const double *q = ((entry_level(jb, i, w) & 2) == 0) ? q0 : q1;
            pp[i] = pressure64(q[i], q[wp + i], q[2 * wp + i]);
        }
    }
    __syncthreads();

    const double lam = jb.coef;
    const double half_lam = 0.5 * lam;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j);
        const int lo = a + 1, hi = w - a + 1;  // active LDS indices [lo, hi)
        const int t = (int)((jb.base + j - 1) & 3);
        if ((t & 1) == 0) {
            for (int i = lo + tid; i < hi; i += NT)
                pr[i] = ratio(pp[i - 1], pp[i], pp[i + 1]);
        } else {
            // predictor (t = 1) reads Q0 and writes Q1, corrector (t = 3)
            // reads Q1 and updates Q0: no lane reads what another writes
            const double *q = (t == 1) ? q0 : q1;
            double *dst = (t == 1) ? q1 : q0;
            const double c = (t == 1) ? half_lam : lam;
            const int chunks = (hi - lo + kFaceLanes - 1) / kFaceLanes;
            for (int k = wave; k < chunks; k += kWaves) {
                const int cell = lo + kFaceLanes * k + lane;
                const int i = cell < hi ? cell : hi;  // face between LDS cells i-1 and i
                double f0, f1, f2;
                face64(q[i - 1], q[wp + i - 1], q[2 * wp + i - 1], q[i], q[wp + i], q[2 * wp + i],
                       pr[i - 1], pr[i], f0, f1, f2);
                const double g0 = from_next_lane(f0);
                const double g1 = from_next_lane(f1);
                const double g2 = from_next_lane(f2);
                if (lane < kFaceLanes && cell < hi) {
                    const double n0 = q0[cell] + c * (f0 - g0);
                    const double n1 = q0[wp + cell] + c * (f1 - g1);
                    const double n2 = q0[2 * wp + cell] + c * (f2 - g2);
                    dst[cell] = n0;
                    dst[wp + cell] = n1;
                    dst[2 * wp + cell] = n2;
                    pp[cell] = pressure64(n0, n1, n2);
                }
            }
        }
        __syncthreads();
    }

    for (int i = 1 + tid; i <= w; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            for (int k = 0; k < 3; ++k)
                state[k * n + g] = q0[k * wp + i];
        } else {
            for (int k = 0; k < 7; ++k)
                ws_out[k * n + g] = lds[k * wp + i];
        }
    }
}

// ---- binary32 with binary64 islands ------------------------------------------

__host__ __device__ __forceinline__ double pressure32(float rho, float m, float e)
{
    const double dr = (double)rho, dm = (double)m, de = (double)e;
    const double u = dm / dr;
    return kGm1 * (de - 0.5 * (dm * u));
}

__host__ __device__ __forceinline__ void face32(float a0, float a1, float a2, float b0, float b1, float b2,
                                       double pra, double prb, float &f0, float &f1, float &f2)
{
    const float hl = 0.5f * (float)limiter(1.0 / pra);
    const float hr = 0.5f * (float)limiter(prb);
    const float d0 = b0 - a0, d1 = b1 - a1, d2 = b2 - a2;
    const float l0 = a0 + hl * d0, l1 = a1 + hl * d1, l2 = a2 + hl * d2;
    const float r0 = b0 - hr * d0, r1 = b1 - hr * d1, r2 = b2 - hr * d2;
    const double rl = (double)l0, ml = (double)l1, el = (double)l2;
    const double rr = (double)r0, mr = (double)r1, er = (double)r2;
    RnDiv dl, dr;
    const double vl64 = rn_div_keep(ml, rl, dl), vr64 = rn_div_keep(mr, rr, dr);
    const double pl64 = kGm1 * (el - 0.5 * (ml * vl64));
    const double pr64 = kGm1 * (er - 0.5 * (mr * vr64));
    double al64, ar64;
    rn_sqrt2(rn_div_again(kGamma * pl64, dl), rn_div_again(kGamma * pr64, dr), al64, ar64);
    const float vl = (float)vl64, pl = (float)pl64, al = (float)al64;
    const float vr = (float)vr64, pr = (float)pr64, ar = (float)ar64;
    const float sl = fabsf(vl) + al;
    const float sr = fabsf(vr) + ar;
    const float hs = 0.5f * (sl > sr ? sl : sr);
    f0 = 0.5f * (l1 + r1) - hs * (r0 - l0);
    f1 = 0.5f * ((l1 * vl + pl) + (r1 * vr + pr)) - hs * (r1 - l1);
    f2 = 0.5f * ((l2 + pl) * vl + (r2 + pr) * vr) - hs * (r2 - l2);
}

__host__ __device__ __forceinline__ float kahan_add(float q, float d, float &c)
{
    const float y = d - c;
    const float t = q + y;
    c = (t - q) - y;
    return t;
}

// LDS: pr[wp], P[wp] (double), q0[3][wp], c[3][wp], q1[3][wp] (float).
// ws layout: q0[3][n], c[3][n], q1[3][n] floats, then pr[n] doubles at byte 36n.
template <int NT, int WT = 0>
__device__ __forceinline__ void euler_f32_tile(const TileJob &jb, double *ldsd)
{
    const int w = WT > 0 ? WT : jb.w;  // compile-time width when WT > 0
    const int wp = w + 2;
    constexpr int kWaves = NT / 64;
    const int64_t n = jb.n;
    double *pr = ldsd;
    double *pp = ldsd + wp;
    float *fst = (float *)(ldsd + 2 * wp);  // q0[3], c[3], q1[3]
    float *q0 = fst;
    float *cc = fst + 3 * wp;
    float *q1 = fst + 6 * wp;
    float *state = (float *)jb.state;
    const float *win = (const float *)jb.ws_in;
    const double *win_pr = (const double *)((const char *)jb.ws_in + 36 * n);
    float *wout = (float *)jb.ws_out;
    double *wout_pr = (double *)((char *)jb.ws_out + 36 * n);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid) >> 6;

    for (int i = tid; i < wp; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.first) {
            for (int k = 0; k < 6; ++k)
                fst[k * wp + i] = state[k * n + g];
            pp[i] = pressure32(q0[i], q0[wp + i], q0[2 * wp + i]);
        } else {
            for (int k = 0; k < 9; ++k)
                fst[k * wp + i] = win[k * n + g];
            pr[i] = win_pr[g];
            const float *q = ((entry_level(jb, i, w) & 2) == 0) ? q0 : q1;
            pp[i] = pressure32(q[i], q[wp + i], q[2 * wp + i]);
        }
    }
    __syncthreads();

    const float lam = (float)jb.coef;
    const float half_lam = 0.5f * lam;
    for (int j = jb.j_first; j <= jb.j_last; ++j) {
        const int a = window_margin(j);
        const int lo = a + 1, hi = w - a + 1;
        const int t = (int)((jb.base + j - 1) & 3);
        if ((t & 1) == 0) {
            for (int i = lo + tid; i < hi; i += NT)
                pr[i] = ratio(pp[i - 1], pp[i], pp[i + 1]);
        } else {
            const float *q = (t == 1) ? q0 : q1;
            const int chunks = (hi - lo + kFaceLanes - 1) / kFaceLanes;
            for (int k = wave; k < chunks; k += kWaves) {
                const int cell = lo + kFaceLanes * k + lane;
                const int i = cell < hi ? cell : hi;
                float f0, f1, f2;
                face32(q[i - 1], q[wp + i - 1], q[2 * wp + i - 1], q[i], q[wp + i], q[2 * wp + i],
                       pr[i - 1], pr[i], f0, f1, f2);
                const float g0 = from_next_lane(f0);
                const float g1 = from_next_lane(f1);
                const float g2 = from_next_lane(f2);
                if (lane < kFaceLanes && cell < hi) {
                    float nq[3];
                    const float f[3] = {f0, f1, f2}, gg[3] = {g0, g1, g2};
                    if (t == 1) {
                        for (int m = 0; m < 3; ++m) {
                            nq[m] = q0[m * wp + cell] + half_lam * (f[m] - gg[m]);
                            q1[m * wp + cell] = nq[m];
                        }
                    } else {
                        for (int m = 0; m < 3; ++m) {
                            float comp = cc[m * wp + cell];
                            nq[m] = kahan_add(q0[m * wp + cell], lam * (f[m] - gg[m]), comp);
                            cc[m * wp + cell] = comp;
                            q0[m * wp + cell] = nq[m];
                        }
                    }
                    pp[cell] = pressure32(nq[0], nq[1], nq[2]);
                }
            }
        }
        __syncthreads();
    }

    for (int i = 1 + tid; i <= w; i += NT) {
        const int64_t g = wrap_cell(jb.g0 + i, n);
        if (jb.last) {
            for (int k = 0; k < 6; ++k)
                state[k * n + g] = fst[k * wp + i];
        } else {
            for (int k = 0; k < 9; ++k)
                wout[k * n + g] = fst[k * wp + i];
            wout_pr[g] = pr[i];
        }
    }
}

} // namespace sw
