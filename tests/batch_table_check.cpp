// Host check of the batch item numbering (csrc/batch.h, csrc/batch_plan.h),
// built with g++ by tests/test_batch_schedule.py.  For random problem lists
// it plans the table and resolves every item number, then checks that the
// numbering is a bijection onto (problem, phase, tile), that phases never
// decrease along the numbering (every dependency has a smaller number) and
// that the item count is the sum of tiles x item phases.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "batch_plan.h"

static uint64_t g_rng = 0x243F6A8885A308D3ull;
static int rnd(int lo, int hi)  // inclusive
{
    g_rng = g_rng * 6364136223846793005ull + 1442695040888963407ull;
    return lo + (int)((g_rng >> 33) % (uint64_t)(hi - lo + 1));
}

static int check(const std::vector<sw::BatchProblem> &in)
{
    sw::BatchPlan plan;
    if (!sw::plan_batch(in, &plan)) {
        fprintf(stderr, "plan overflow\n");
        return 1;
    }
    const int n = (int)in.size();
    int64_t expect = 0;
    for (const auto &p : in)
        expect += (int64_t)p.tiles * p.item_phases;
    if (plan.n_items != expect) {
        fprintf(stderr, "items %lld != %lld\n", (long long)plan.n_items, (long long)expect);
        return 1;
    }
    std::vector<std::vector<char>> seen(n);
    for (int s = 0; s < n; ++s) {
        if (in[plan.order[s]].tiles != plan.table[s].tiles) {
            fprintf(stderr, "order mismatch\n");
            return 1;
        }
        if (s > 0 && plan.table[s - 1].item_phases < plan.table[s].item_phases) {
            fprintf(stderr, "table not sorted\n");
            return 1;
        }
        seen[s].assign((size_t)plan.table[s].tiles * plan.table[s].item_phases, 0);
    }
    int last_phase = 1;
    for (int64_t item = 0; item < plan.n_items; ++item) {
        const sw::BatchItem it = sw::batch_item(plan.table.data(), n, item);
        if (it.problem < 0 || it.problem >= n) {
            fprintf(stderr, "item %lld: problem %d\n", (long long)item, it.problem);
            return 1;
        }
        const sw::BatchProblem &p = plan.table[it.problem];
        if (it.phase < 1 || it.phase > p.item_phases || it.tile < 0 || it.tile >= p.tiles) {
            fprintf(stderr, "item %lld: phase %d tile %d out of range\n", (long long)item, it.phase,
                    it.tile);
            return 1;
        }
        if (it.phase < last_phase) {
            fprintf(stderr, "item %lld: phase decreases\n", (long long)item);
            return 1;
        }
        last_phase = it.phase;
        char &c = seen[it.problem][(size_t)(it.phase - 1) * p.tiles + it.tile];
        if (c) {
            fprintf(stderr, "item %lld: duplicate\n", (long long)item);
            return 1;
        }
        c = 1;
    }
    return 0;  // every slot was hit: counts match and no duplicate
}

int main(int argc, char **argv)
{
    const int cases = argc > 1 ? atoi(argv[1]) : 300;
    for (int c = 0; c < cases; ++c) {
        const int n = c < 3 ? 1 + c : rnd(1, 40);
        const bool equal = (c % 7) == 3;  // every problem with the same phase count
        std::vector<sw::BatchProblem> in(n);
        for (int i = 0; i < n; ++i) {
            in[i] = sw::BatchProblem{};
            in[i].tiles = rnd(2, 17);
            in[i].item_phases = equal ? 5 : rnd(1, 30);
        }
        if (check(in)) {
            fprintf(stderr, "case %d failed\n", c);
            return 1;
        }
    }
    printf("ok %d cases\n", cases);
    return 0;
}
