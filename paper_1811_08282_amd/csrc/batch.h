// batch.h -- device tables of the persistent batched swept launch.
//
// Work items are (problem p, phase k, tile t).  They are numbered phase by
// phase (all problems' phase-1 tiles, then all phase-2 tiles, ...), so every
// item's dependencies carry smaller numbers.  A global ticket hands items out
// in that order; an item waits until the two tiles of the previous phase that
// overlap its cells have published completion flags, runs the tile-phase
// body, then publishes its own flag.
//
// Dependencies of phase k > 1, tile t (tiles of phase k start at offset 0
// for odd k and W/2 for even k; halos of R <= W/2 cells):
//   k even: previous-phase tiles t and t+1;  k odd: t-1 and t   (mod tiles)
// Those two tiles are the only previous-phase tiles that write cells this
// tile reads (its W cells and both halos) and the only ones that read cells
// of the working array this tile overwrites, so both the read-after-write and
// the write-after-read orders are covered.
//
// A problem with a single phase (heat, one step) gets a copy-out item per
// tile as phase 2: it copies its tile's cells from the working array to the
// state once tiles t-1, t and t+1 of phase 1 (the readers of those cells)
// are done.
#pragma once

#include <stdint.h>

#include "geom.h"

namespace sw {

struct BatchProblem {
    void *state;
    void *ws0;             // working arrays written by odd phases
    void *ws1;             // working arrays written by even phases
    int64_t n;
    int64_t final_level;
    int64_t phases;        // schedule phases K (copy-out adds one item phase)
    int64_t flag_off;      // index of tile 0's flag
    double coef;           // r (heat) or lambda (Euler)
    int w;
    int eq;                // sw_equation
    int tiles;
    int single_phase;      // K == 1
    int radius;            // stencil radius of one sub-step (2: flattened Euler)
};

struct BatchSegment {
    int64_t start;         // first item number
    int problem;
    int phase;
};

struct BatchTables {
    const BatchProblem *problems;
    const BatchSegment *segments;
    int64_t n_segments;
    int64_t n_items;
    unsigned long long *ticket;
    int *flags;
    int *status;           // 0 ok; 1 a dependency wait exceeded its time bound
    long long wait_limit;  // bound of one dependency wait, in s_memrealtime ticks
};

// previous-phase tiles an item depends on (count returned; at most 3)
SW_HD int batch_deps(int phase, int tile, int tiles, int single_phase,
                                          int deps[3])
{
    if (phase <= 1)
        return 0;
    const int prev = (tile - 1 + tiles) % tiles;
    const int next = (tile + 1) % tiles;
    if (single_phase) {
        deps[0] = prev;
        deps[1] = tile;
        deps[2] = next;
        return 3;
    }
    if (phase % 2 == 0) {
        deps[0] = tile;
        deps[1] = next;
    } else {
        deps[0] = prev;
        deps[1] = tile;
    }
    return 2;
}

} // namespace sw
