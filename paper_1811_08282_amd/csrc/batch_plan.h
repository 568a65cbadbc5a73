// batch_plan.h -- host planner of the batch table (batch.h): sorts the
// problems by item phases, assigns flag offsets and item blocks, and counts
// the items.  Host only; no HIP call.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "batch.h"

namespace sw {

struct BatchPlan {
    std::vector<BatchProblem> table;  // sorted by item_phases, descending (stable)
    std::vector<int> order;           // table index -> caller's problem index
    int64_t n_items = 0;
    int64_t n_flags = 0;              // tiles of every problem
};

// `in` holds one entry per problem in the caller's order with every field
// set except flag_off and item_block.  Returns false when the item count
// overflows 64 bits.
inline bool plan_batch(const std::vector<BatchProblem> &in, BatchPlan *out)
{
    const int n = (int)in.size();
    out->order.resize(n);
    std::iota(out->order.begin(), out->order.end(), 0);
    std::stable_sort(out->order.begin(), out->order.end(),
                     [&](int a, int b) { return in[a].item_phases > in[b].item_phases; });
    out->table.resize(n);
    int64_t tiles = 0;
    for (int s = 0; s < n; ++s) {
        BatchProblem p = in[out->order[s]];
        p.flag_off = tiles;
        tiles += p.tiles;
        out->table[s] = p;
    }
    int64_t start = 0;
    for (int s = n - 1; s >= 0; --s) {
        BatchProblem &p = out->table[s];
        p.item_block = start;
        const int64_t below = s + 1 < n ? out->table[s + 1].item_phases : 0;
        const int64_t phases = p.item_phases - below;
        const int64_t per_phase = p.flag_off + p.tiles;
        int64_t items = 0;
        if (__builtin_mul_overflow(phases, per_phase, &items) ||
            __builtin_add_overflow(start, items, &start))
            return false;
    }
    out->n_items = start;
    out->n_flags = tiles;
    return true;
}

} // namespace sw
