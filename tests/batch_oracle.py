"""Oracle side of the full-size batch test (4096 problems x 5000 steps).

The test checks 128 problems of the batch against the oracle.  Stepping
their dependency cones on the host takes minutes, so the oracle values are
computed once by tests/golden/make_batch_oracle.py (which calls only
oracle/) and stored as SHA-256 digests in tests/golden/batch_oracle.json;
the GPU test compares the digest of its own values with them and re-steps
the two widest problems live.  Everything here is numpy and the oracle.
"""
import hashlib
import json
import os

import numpy as np

import oracle
import paper_1811_08282_amd as sw
from paper_1811_08282_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_oracle.json")
STEPS = 5000
# precision pairs of the batched workload: (heat id, Euler id)
PAIRS = {"f64": (sw.HEAT_F64, sw.EULER_F64), "f32": (sw.HEAT_F32, sw.EULER_F32)}

# cells a cell's value after one time step depends on, per side: heat 1;
# Euler 4 (the corrector reads the predictor within 2 cells, which read the
# old state within 2)
CONE = {sw.HEAT_F64: 1, sw.HEAT_F32: 1, sw.EULER_F64: 4, sw.EULER_F32: 4}


def pack(eq, q):
    """numpy initial state -> array of shape (rows, n) in the eq's layout."""
    if sw.is_f64(eq):
        return np.array(q, dtype=np.float64, copy=True).reshape(sw.state_rows(eq), -1)
    q32 = np.asarray(q, dtype=np.float32).reshape(-1, np.asarray(q).shape[-1])
    return np.concatenate([q32, np.zeros_like(q32)])


def problems(pair):
    """(problems, ids, host initial states) of the batched workload."""
    eq_heat, eq_euler = PAIRS[pair]
    probs = wl.batch_problems()
    ids = [eq_heat if p.eq == "heat" else eq_euler for p in probs]
    hosts = [pack(e, wl.batch_ic(p)) for e, p in zip(ids, probs)]
    return probs, ids, hosts


def subset(probs, count=128, seed=128):
    """`count` problems drawn across the length range: the problems sorted by
    length are cut into `count` strata of equal size and one problem is drawn
    from each (seeded); the longest heat and the longest Euler problem (the
    widest tiles the tuner picks) replace the draws of the last two strata."""
    rng = np.random.default_rng(seed)
    order = np.argsort([p.n for p in probs], kind="stable")
    strata = np.array_split(order, count)
    pick = [int(rng.choice(s)) for s in strata]
    longest_heat = max((i for i, p in enumerate(probs) if p.eq == "heat"), key=lambda i: probs[i].n)
    longest_euler = max((i for i, p in enumerate(probs) if p.eq != "heat"),
                        key=lambda i: probs[i].n)
    pick[-2:] = [longest_heat, longest_euler]
    return sorted(set(pick))


def sample_cells(eq, n, steps=STEPS):
    """Cells of a problem the oracle values cover: all of them when the
    problem is no longer than its dependency cone, else 16 cells straddling
    the periodic seam."""
    reach = CONE[eq] * steps + 4
    if n <= 2 * reach + 64:
        return np.arange(n)
    return (np.arange(n - 8, n + 8)) % n


def sample(eq, host, steps=STEPS, threads=0):
    """Oracle values of one problem at sample_cells: the whole problem, or
    the 16 cells stepped from the exact cone around them (2 * cone * steps
    + 16 cells, a ring whose own wrap cannot reach the centre).  Returns
    (cells, values) with values shaped like host[:, cells]."""
    n = host.shape[1]
    cells = sample_cells(eq, n, steps)
    reach = CONE[eq] * steps + 4
    if cells.size == n:
        idx, keep = np.arange(n), slice(0, n)
    else:
        s0 = n - 8
        idx, keep = np.arange(s0 - reach, s0 + 16 + reach) % n, slice(reach, reach + 16)
    h = host[:, idx]
    if eq == sw.HEAT_F64:
        out = oracle.heat_f64(h[0], steps, 0.25, threads=threads).reshape(1, -1)
    elif eq == sw.EULER_F64:
        out = oracle.euler_f64(h, steps, 0.1, threads=threads)
    elif eq == sw.HEAT_F32:
        out = np.stack(oracle.heat_f32(h[0], h[1], steps, 0.25, threads=threads))
    else:
        q, c = oracle.euler_f32(h[:3], h[3:], steps, 0.1, threads=threads)
        out = np.concatenate([q, c])
    return cells, np.ascontiguousarray(out[:, keep])


def digest(values):
    """SHA-256 of the values' bytes, with their dtype and shape."""
    v = np.ascontiguousarray(values)
    h = hashlib.sha256(f"{v.dtype.str}{v.shape}".encode())
    h.update(v.tobytes())
    return h.hexdigest()


def load_golden():
    with open(GOLDEN) as f:
        return json.load(f)
