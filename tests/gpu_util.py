"""Helpers shared by the GPU tests: device round trips through the C ABI."""
import json
import os
import sys

import numpy as np

import paper_1811_08282_amd as sw


def announce(*parts):
    """Name the GPU case about to run (flushed, so a fault still leaves it)."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def pack(eq, q):
    """numpy initial state -> host array of shape (rows, n) in the eq's dtype.

    heat: q has shape (n,); Euler: (3, n).  F32 states get zero compensations.
    """
    q = np.asarray(q, dtype=np.float64)
    if eq == sw.HEAT_F64:
        return q.reshape(1, -1).copy()
    if eq == sw.HEAT_F32:
        return np.stack([q.astype(np.float32), np.zeros(q.shape, np.float32)])
    if eq == sw.EULER_F64:
        return q.copy()
    return np.concatenate([q.astype(np.float32), np.zeros(q.shape, np.float32)])


def run(eq, host_state, steps, dt, dx, method="swept", width=0, chunks=None, threads=0):
    """Upload, solve (optionally as several calls), download."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(host_state)).cuda()
    for part in (chunks or [steps]):
        sw.solve(eq, t, part, dt, dx, method=method, width=width, threads=threads)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_inf(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den else float(np.max(np.abs(a - b)))


def record(name, **values):
    """Print a measured figure (e.g. an error against the oracle) and append
    it as one JSON line to the file named by SWEPT_RECORD_FILE, if set."""
    line = json.dumps(dict(name=name, **values))
    print("[measured]", line, flush=True)
    path = os.environ.get("SWEPT_RECORD_FILE")
    if path:
        with open(path, "a") as f:
            f.write(line + "\n")
