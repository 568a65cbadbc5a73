// batch.h -- device table of the persistent batched swept launch.
//
// Work items are (problem, phase k, tile t).  They are numbered phase by
// phase (every problem's phase-1 tiles, then every phase-2 tile, ...), so
// every item's dependencies carry smaller numbers.  A global ticket hands
// items out in that order; an item waits until the two tiles of the previous
// phase that overlap its cells have published completion flags, runs the
// tile-phase body, then publishes its own flag.
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
//
// Item numbering without a per-phase table.  The problems are stored sorted
// by their number of item phases P (schedule phases plus the copy-out phase)
// in descending order, so the problems active in phase k are a prefix of the
// table: the first A(k) = #{s : P_s >= k}.  A(k) changes only where k passes
// some P_s, so the items split into at most n blocks; block s holds the
// phases P_{s+1} + 1 .. P_s (P_n = 0), in each of which exactly the problems
// 0..s are active, tile after tile in table order.  With TP(a) the tiles of
// the first a problems (the flag offset of problem a), block s starts at
//     B_{n-1} = 0,   B_{s-1} = B_s + (P_s - P_{s+1}) * TP(s+1),
// and the item count is B_{-1}.  An item number is resolved by two binary
// searches over the table (batch_item), so the table has n entries whatever
// the number of phases.
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
    int64_t flag_off;      // index of tile 0's flag = tiles of the problems before it
    int64_t item_block;    // B_s: first item of the block whose last active problem this is
    double coef;           // r (heat) or lambda (Euler)
    int w;
    int eq;                // sw_equation
    int tiles;
    int single_phase;      // K == 1
    int radius;            // stencil radius of one sub-step (2: flattened Euler)
    int item_phases;       // P = K + single_phase
};

struct BatchTables {
    const BatchProblem *problems;  // sorted by item_phases, descending
    int n_problems;
    int64_t n_items;
    unsigned long long *ticket;
    int *flags;
    int *status;           // 0 ok; 1 a dependency wait exceeded its time bound
    long long wait_limit;  // bound of one dependency wait, in s_memrealtime ticks
};

struct BatchItem {
    int problem;           // index in the sorted table
    int phase;             // 1-based item phase
    int tile;
};

// (problem, phase, tile) of item number `item` < n_items
SW_HD BatchItem batch_item(const BatchProblem *p, int n, int64_t item)
{
    // block: the smallest s with B_s <= item (B is non-increasing in s)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (p[mid].item_block <= item)
            hi = mid;
        else
            lo = mid + 1;
    }
    const int s = lo;
    const int64_t rel = item - p[s].item_block;
    const int64_t per_phase = p[s].flag_off + p[s].tiles;  // TP(s + 1)
    const int64_t below = (s + 1 < n) ? p[s + 1].item_phases : 0;
    BatchItem r;
    r.phase = (int)(below + 1 + rel / per_phase);
    const int64_t o = rel % per_phase;
    // problem: the largest j <= s with flag_off_j <= o
    int a = 0, b = s;
    while (a < b) {
        const int mid = (a + b + 1) / 2;
        if (p[mid].flag_off <= o)
            a = mid;
        else
            b = mid - 1;
    }
    r.problem = a;
    r.tile = (int)(o - p[a].flag_off);
    return r;
}

// previous-phase tiles an item depends on (count returned; at most 3)
SW_HD int batch_deps(int phase, int tile, int tiles, int single_phase, int deps[3])
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
