// geom.h -- geometry of the swept schedule, shared by the host planner and
// the phase kernels.
//
// Written here for a three-point stencil (radius R = 1).  A sub-step of
// radius R (the five-point "flattened" Euler sub-steps have R = 2) scales
// every margin by R: H = W / (2R) levels per half phase, windows
// [R|j - 1|, W - R|j - 1|), R halo cells per side; the tiling still shifts by
// W/2 between phases.
//
// Sub-step levels: level 0 is the initial state, level m the state after m
// sub-steps; the run ends at level F.  With tile width W = 2H the schedule
// has K phases (Sec. 4.1): phase 1 is the Up Triangle, phases 2..K-1 the
// Diamonds, phase K the Down Triangle.  Odd phases tile the grid from cell 0,
// even phases from cell H, so each tile of an even phase is centred on a
// seam of the odd tiling and the other way round -- the alternating edge
// exchange of the paper becomes a shift of the tiling by H.
//
// Inside a tile of phase k, with base = (k - 1) H and relative level
// j = m - base, the cells that compute level m are
//     o in [|j - 1|, W - |j - 1|)           (tile coordinates, o in [0, W))
// for j in [j_first, j_last], j_first = 1 for k = 1 and 2 - H otherwise,
// j_last = min(H, F - base).  Read from the bottom: the window widens by one
// cell per side per level while the void left by the previous phase is
// filled (j <= 1), then narrows by one cell per side while the next triangle
// is built (j >= 1): W^2 / 2 cell-levels per full Diamond, none repeated.
//
// Every level of a tile needs, besides its W cells, one cell on each side
// (halo) only at j = 1, and then at level base, the peak level of the
// previous phase.  Each cell enters a phase with its two most recent levels
// and leaves with its two most recent levels, which is what the two-slot
// working struct holds.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define SW_HD __host__ __device__ inline
#else
#define SW_HD inline
#endif

namespace sw {

SW_HD int64_t phase_count(int64_t final_level, int64_t half)
{
    if (final_level <= 0)
        return 0;
    return (final_level - 1 + half - 1) / half + 1;
}

struct PhaseRange {
    int64_t base;    // (k - 1) * H
    int64_t offset;  // first cell of tile 0
    int j_first;     // first relative level
    int j_last;      // last relative level (j_first > j_last: nothing to do)
};

// `half` = H, levels per half phase (W / 2R); `radius` = R
SW_HD PhaseRange phase_range(int64_t k, int64_t final_level, int64_t half, int radius = 1)
{
    PhaseRange p;
    p.base = (k - 1) * half;
    p.offset = ((k - 1) & 1) ? half * radius : 0;
    p.j_first = (k == 1) ? 1 : (int)(2 - half);
    int64_t top = final_level - p.base;
    p.j_last = (int)(top < half ? top : half);
    return p;
}

// distance of the active window from each tile edge at relative level j
SW_HD int window_margin(int j, int radius = 1)
{
    return radius * (j >= 1 ? j - 1 : 1 - j);
}

} // namespace sw
