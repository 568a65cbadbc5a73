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
// struct (slot m & 1 holds level m), the phase's levels are swept (below),
// and the W owned cells are written back.
//
// Level sweep, register blocked.  The levels of a phase are taken in blocks
// of kRbL levels, never mixing the part where the window widens (j <= 1) with
// the part where it narrows.  A block reads the cells of its widest window
// from LDS into registers, advances them kRbL levels without touching LDS and
// writes them back, with two barriers per block instead of one per level:
//  * a row is one wave: each lane holds kRbC consecutive cells, both level
//    parities of each, and takes the neighbours of its end cells from the
//    adjacent lanes by DPP shifts;
//  * lanes 0 and 63 of a row are ghosts holding copies of the next row's
//    cells; the values of lanes 1..62 stay exact for kRbC >= kRbL levels, so
//    rows never exchange data inside a block;
//  * row 0 starts at the window's left edge and the last row ends at its
//    right edge, its lanes running downward (lane 1 holds the rightmost
//    cells); in these two edge rows the cells outside the window at a level
//    keep their values (the ghost cell next to the window, and the first
//    cells of lane 1), which is all the window edge needs; every other row
//    runs unmasked;
//  * each cell is written back by exactly one row: the upward rows up to a
//    split point, the downward row from there, both at least 2 kRbL cells
//    from the window edge they do not mask (a lane's values can only go wrong
//    within kRbL cells of an unmasked edge, spreading one cell per level).
// Windows too narrow for two rows of this shape are swept level by level in
// LDS (one barrier per level).
#pragma once

#include "geom.h"
#include "lanes.h"
#include "tile_job.h"

namespace sw {

__host__ __device__ __forceinline__ double heat_update(double l, double c, double r_, double r)
{
    return c + r * ((r_ - c) + (l - c));
}

__host__ __device__ __forceinline__ float heat_update_kahan(float l, float c, float rr, float r, float &comp)
{
    const float d = r * ((rr - c) + (l - c));
    const float y = d - comp;
    const float t = c + y;
    comp = (t - c) - y;
    return t;
}

constexpr int kRbC = 5;        // consecutive cells per lane (a 40-byte lane stride: no LDS bank conflicts)
constexpr int kRbL = 5;        // levels per register block (<= kRbC)
constexpr int kRbOwned = 62;   // lanes of a row whose cells it owns (1..62)
constexpr int kRbRows = 2;     // rows held per wave
static_assert(kRbL <= kRbC, "ghost lanes must cover the levels of a block");
static_assert(kHeatLdsPad >= kRbC, "LDS padding must cover a ghost lane beyond the halo");

// one level sweep of the LDS window, cells [a + 1, w - a] (LDS indices)
template <typename T, bool KAHAN, int NT>
__device__ __forceinline__ void heat_level_lds(T *s0, T *s1, T *cc, int w, int64_t m, int a, T r)
{
    const T *src = (m & 1) ? s0 : s1;
    T *dst = (m & 1) ? s1 : s0;
    const int end = w - a;
    int i = a + 1 + (int)threadIdx.x;
    if constexpr (KAHAN) {
        // two cells per thread and pass (i and i + NT): their LDS accesses pair
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
    } else {
        for (; i <= end; i += NT)
            dst[i] = heat_update(src[i - 1], src[i], src[i + 1], r);
    }
    __syncthreads();
}

// Rows of one block.  Outer window [e_lo, e_hi] (LDS indices); q lanes of
// kRbC cells from e_lo end at the split sp; rows 0..rows-2 start at
// e_lo + 62 kRbC r (lanes upward), row rows-1 ends at e_hi (lanes downward).
struct RbGeom {
    int e_lo, e_hi, sp, rows;
};

__device__ __forceinline__ bool rb_plan(int w, int a_out, int slots, RbGeom &g)
{
    g.e_lo = a_out + 1;
    g.e_hi = w - a_out;
    const int wo = g.e_hi - g.e_lo + 1;
    // the downward row writes at most 62 lanes, and nothing within 2L of
    // the left edge; the upward rows write nothing within 2L of the right edge
    constexpr int qmin = (2 * kRbL + kRbC - 1 + kRbC - 1) / kRbC;
    int q = (wo + kRbC - 1) / kRbC - kRbOwned;
    if (q < qmin)
        q = qmin;
    g.rows = 1 + (q + kRbOwned - 1) / kRbOwned;
    g.sp = g.e_lo + kRbC * q;
    return kRbC * q <= wo - 1 - 2 * kRbL && g.rows <= slots;
}

// One level of one row: lane values v[parity][cell] (cells in ascending LDS
// order), Kahan compensations k.  Writes parity Q from parity Q ^ 1.  The
// update is evaluated with one difference per face, D[j] = u(j) - u(j - 1):
//     u' = u + r * (D[c + 1] - D[c])
// which equals u + r * ((u_right - u) + (u_left - u)) bit for bit: IEEE
// subtraction is sign-symmetric, so u_left - u == -D[c] whenever it is not
// zero, a + (-b) == a - b, and the one signed-zero case where the sums
// differ (u == +0, u_left == +0, u_right == -0) gives u' == +0 either way.
// DOWN: the row's lanes run downward (lane l + 1 holds the cells below).  In
// an edge row the ghost cell next to the window and the cells of lane 1 not
// yet or no longer in the window (`frz` of them, counted from the edge) keep
// their values.
template <typename T, bool KAHAN, int Q, bool DOWN, bool EDGE>
__device__ __forceinline__ void rb_level(T (&v)[2][kRbC], T (&k)[kRbC], int frz, int lane, T r)
{
    constexpr int QR = Q ^ 1;
    const T below = DOWN ? from_next_lane(v[QR][kRbC - 1]) : from_prev_lane(v[QR][kRbC - 1]);
    const T above = DOWN ? from_prev_lane(v[QR][0]) : from_next_lane(v[QR][0]);
    T d[kRbC + 1];
    d[0] = v[QR][0] - below;
#pragma unroll
    for (int c = 1; c < kRbC; ++c)
        d[c] = v[QR][c] - v[QR][c - 1];
    d[kRbC] = above - v[QR][kRbC - 1];
#pragma unroll
    for (int c = 0; c < kRbC; ++c) {
        const T inc = r * (d[c + 1] - d[c]);
        T nv, nk;
        if constexpr (KAHAN) {
            const T y = inc - k[c];
            nv = v[QR][c] + y;
            nk = (nv - v[QR][c]) - y;
        } else {
            nv = v[QR][c] + inc;
            nk = T(0);
        }
        if constexpr (EDGE) {
            // cells that can keep their value at this level: lane 0's cell
            // next to the window, and lane 1's frozen cells
            const bool ghost = DOWN ? c == 0 : c == kRbC - 1;
            const bool frozen = DOWN ? c >= kRbC - frz : c < frz;
            if (ghost || frozen) {
                const bool keep = (ghost && lane == 0) || (frozen && lane == 1);
                v[Q][c] = keep ? v[Q][c] : nv;
                if constexpr (KAHAN)
                    k[c] = keep ? k[c] : nk;
                continue;
            }
        }
        v[Q][c] = nv;
        if constexpr (KAHAN)
            k[c] = nk;
    }
}

template <typename T, bool KAHAN, int Q>
__device__ __forceinline__ void rb_level_row(T (&v)[2][kRbC], T (&k)[kRbC], int f, int frz,
                                             int lane, T r)
{
    if (f == 0)
        rb_level<T, KAHAN, Q, false, true>(v, k, frz, lane, r);
    else if (f == 1)
        rb_level<T, KAHAN, Q, true, true>(v, k, frz, lane, r);
    else
        rb_level<T, KAHAN, Q, false, false>(v, k, frz, lane, r);
}

// Levels j in [ja, jz] (at most kRbL, all with j <= 1 when WID, all with
// j >= 2 otherwise).  Register parity 0 holds LDS slot p0, the parity of the
// block's virtual first level; virtual level t of the block writes parity
// t & 1.  WID is a template argument so that, with the level loop unrolled,
// the number of frozen edge cells at each level is a constant and only the
// cells that can freeze cost a select.
template <typename T, bool KAHAN, int NT, bool WID>
__device__ __forceinline__ void heat_rb_block(T *s0, T *s1, T *cc, int w, int64_t base, int ja,
                                              int jz, T r)
{
    constexpr int NW = NT / 64;
    constexpr bool wid = WID;
    const int nl = jz - ja + 1;
    const int a_out = wid ? 1 - jz : ja - 1;
    const int t_lo = wid ? kRbL - nl : 0;
    const int t_hi = wid ? kRbL : nl;
    const int64_t jv0 = wid ? (int64_t)jz - (kRbL - 1) : (int64_t)ja;
    RbGeom g;
    if (!rb_plan(w, a_out, NW * kRbRows, g)) {
        for (int j = ja; j <= jz; ++j)
            heat_level_lds<T, KAHAN, NT>(s0, s1, cc, w, base + j, window_margin(j), r);
        return;
    }
    const int p0 = (int)((base + jv0) & 1);
    T *sa = p0 ? s1 : s0;
    T *sb = p0 ? s0 : s1;
    const int lane = (int)(threadIdx.x & 63);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));

    // slot s of this wave holds row f = s * NW + wave in the order: the
    // left edge row, the right edge row (lanes downward), the inner rows
    T v[kRbRows][2][kRbC];
    T k[kRbRows][kRbC];
    int lo[kRbRows];  // first LDS index of this lane's cells
    bool wr[kRbRows]; // this lane writes its cells back
#pragma unroll
    for (int s = 0; s < kRbRows; ++s) {
        const int f = s * NW + wave;
        int start;
        if (f == 1) {
            start = g.e_hi - lane * kRbC + 1;
            wr[s] = lane >= 1 && lane <= kRbOwned && start + kRbC - 1 >= g.sp;
        } else {
            const int row = f == 0 ? 0 : f - 1;
            start = g.e_lo + kRbOwned * kRbC * row + (lane - 1) * kRbC;
            wr[s] = lane >= 1 && lane <= kRbOwned && start < g.sp;
        }
        // lanes far outside the tile read clamped (unused) cells
        start = start < -kHeatLdsPad ? -kHeatLdsPad : start;
        start = start > w + 2 + kHeatLdsPad - kRbC ? w + 2 + kHeatLdsPad - kRbC : start;
        lo[s] = start;
        if (f < g.rows) {
#pragma unroll
            for (int c = 0; c < kRbC; ++c) {
                v[s][0][c] = sa[start + c];
                v[s][1][c] = sb[start + c];
                if constexpr (KAHAN)
                    k[s][c] = cc[start + c];
            }
        }
    }

#pragma unroll
    for (int t = 0; t < kRbL; ++t) {
        if (t < t_lo || t >= t_hi)
            continue;
        const int frz = wid ? kRbL - 1 - t : t;
#pragma unroll
        for (int s = 0; s < kRbRows; ++s) {
            const int f = s * NW + wave;
            if (f >= g.rows)
                continue;
            if (t & 1)
                rb_level_row<T, KAHAN, 1>(v[s], k[s], f, frz, lane, r);
            else
                rb_level_row<T, KAHAN, 0>(v[s], k[s], f, frz, lane, r);
        }
    }
    __syncthreads();  // every row has read its cells, ghosts included

#pragma unroll
    for (int s = 0; s < kRbRows; ++s) {
        if (s * NW + wave < g.rows && wr[s]) {
#pragma unroll
            for (int c = 0; c < kRbC; ++c) {
                sa[lo[s] + c] = v[s][0][c];
                sb[lo[s] + c] = v[s][1][c];
                if constexpr (KAHAN)
                    cc[lo[s] + c] = k[s][c];
            }
        }
    }
    __syncthreads();
}

// Sweep levels j_first..j_last of a phase: the widening part (j <= 1) in
// blocks aligned to end at its last level, the narrowing part in blocks from
// its first level.
template <typename T, bool KAHAN, int NT>
__device__ __forceinline__ void heat_levels(T *s0, T *s1, T *cc, int w, int64_t base,
                                            int j_first, int j_last, T r)
{
    const int jw = j_last < 1 ? j_last : 1;
    if (j_first <= jw) {
        const int nlev = jw - j_first + 1;
        int sz = nlev % kRbL;
        if (sz == 0)
            sz = kRbL;
        for (int j = j_first; j <= jw; j += sz, sz = kRbL)
            heat_rb_block<T, KAHAN, NT, true>(s0, s1, cc, w, base, j, j + sz - 1, r);
    }
    for (int j = j_first > 2 ? j_first : 2; j <= j_last; j += kRbL) {
        const int jz = j + kRbL - 1 < j_last ? j + kRbL - 1 : j_last;
        heat_rb_block<T, KAHAN, NT, false>(s0, s1, cc, w, base, j, jz, r);
    }
}

// LDS: s0[w+2], s1[w+2] doubles, each with kHeatLdsPad cells of padding on
// both sides.  ws layout: slot0[n], slot1[n].
template <int NT>
__device__ __forceinline__ void heat_f64_tile(const TileJob &jb, double *lds)
{
    const int w = jb.w;
    const int wp = w + 2;
    const int64_t n = jb.n;
    double *s0 = lds + kHeatLdsPad;
    double *s1 = s0 + wp + 2 * kHeatLdsPad;
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

    heat_levels<double, false, NT>(s0, s1, nullptr, w, jb.base, jb.j_first, jb.j_last, jb.coef);

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

// LDS: s0[w+2], s1[w+2], c[w+2] floats, each padded as above.
// ws layout: u0[n], u1[n], c[n].
template <int NT>
__device__ __forceinline__ void heat_f32_tile(const TileJob &jb, float *ldsf)
{
    const int w = jb.w;
    const int wp = w + 2;
    const int64_t n = jb.n;
    const int stride = wp + 2 * kHeatLdsPad;
    float *s0 = ldsf + kHeatLdsPad;
    float *s1 = s0 + stride;
    float *cc = s1 + stride;
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

    heat_levels<float, true, NT>(s0, s1, cc, w, jb.base, jb.j_first, jb.j_last, (float)jb.coef);

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
