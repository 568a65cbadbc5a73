"""Write tests/golden/batch_oracle.json: oracle digests of the 128-problem
subset of the batched workload (4096 problems, 5000 steps), binary64 and
binary32, for tests/test_gpu_fullsize.py.  Calls only the oracle (through
tests/batch_oracle.py) on the seeded inputs of paper_1811_08282_amd.workloads.

    python tests/golden/make_batch_oracle.py [threads]

Takes tens of CPU-minutes; rerun it whenever the oracle, the batched
workload generator or the subset rule changes.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import batch_oracle as bo  # noqa: E402


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    out = {"steps": bo.STEPS, "note": "sha256 of oracle values at sample_cells, per problem",
           "pairs": {}}
    for pair in ("f64", "f32"):
        probs, ids, hosts = bo.problems(pair)
        sub = bo.subset(probs)
        rows = []
        t0 = time.time()
        for k, i in enumerate(sub):
            cells, vals = bo.sample(ids[i], hosts[i], bo.STEPS, threads)
            rows.append({"problem": i, "eq": ids[i], "n": probs[i].n, "cells": int(cells.size),
                         "sha256": bo.digest(vals),
                         "first": [float(x).hex() for x in vals[:, 0]]})
            if k % 16 == 15:
                print(f"{pair}: {k + 1}/{len(sub)} ({time.time() - t0:.0f} s)", flush=True)
        out["pairs"][pair] = {"subset": sub, "problems": rows}
    with open(bo.GOLDEN, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", bo.GOLDEN)


if __name__ == "__main__":
    main()
