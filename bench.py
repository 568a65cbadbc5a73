#!/usr/bin/env python3
"""Benchmark of the swept-rule hot path on one MI355X.

One benchmark step is one full solve of a workload through the C ABI: every
phase of the swept schedule -- Up Triangle, Diamonds, Down Triangle -- over
the whole grid for all its time steps.  The default run measures the
2^24-cell configuration (the largest single-GPU one) in every equation and
precision: the heat equation (FTCS, r = 1/4, seeded random-mode initial
condition) and the Euler equations (Sod tiles of 2^14 cells, dt/dx = 0.1),
binary64 and binary32 + Kahan, the Euler equations in both sub-step layouts,
20000 time steps each.  The headline value is heat binary64; every leg
reports swept and classic (one launch per sub-step) throughput, their ratio,
its sampled error against the oracle and its rooflines.

Heat grids of more than 1024 tiles of 1792 cells or more run as one
persistent launch per solve (the batched launch holding the single problem,
``sw_batch_run``, as ``swept_solve`` does for them), the other workloads one
launch per phase (``swept_solve``), the faster schedule of each on MI355X.  Every timed solve starts from the initial state, restored from a
device copy outside the timed region; times are HIP events on the launch
stream and the reported time is the median over the timed solves.

Prints ONE JSON line.  Inputs are resident in HBM when the timed region
starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_1811_08282_amd as sw  # noqa: E402
from paper_1811_08282_amd import workloads as wl  # noqa: E402

METRIC = "cell-updates/s swept vs naive (FP64, FP32) at stated error; % HBM roofline"
CUS, CLOCK_HZ = 256, 2.4e9
HBM_PEAK_GBS = 8000.0
# published vector peaks (an FMA counts as two flops; the kernels use no FMA
# and no packed math, and every other operation counts as one flop)
VECTOR_PEAK_TFLOPS = {True: 78.6, False: 157.3}  # binary64, binary32
# LDS rates per compute unit and clock measured on gfx950 by a streaming
# microbenchmark (the best width of each direction: ds_read_b128 and
# ds_write_b128); the port is taken to serve reads and writes one at a time
LDS_READ_B_PER_CLK = 150.4
LDS_WRITE_B_PER_CLK = 70.9
WORKLOADS = {
    "heat_f64_large": (wl.HEAT_LARGE, sw.HEAT_F64),
    "heat_f64_small": (wl.HEAT_SMALL, sw.HEAT_F64),
    "euler_f64_large": (wl.EULER_LARGE, sw.EULER_F64),
    "heat_f32_prec": (wl.HEAT_PREC, sw.HEAT_F32),
    "euler_f32_prec": (wl.EULER_PREC, sw.EULER_F32),
    "heat_f64_prec": (wl.HEAT_PREC, sw.HEAT_F64),
    "euler_f64_prec": (wl.EULER_PREC, sw.EULER_F64),
    "euler_f64_flat_large": (wl.EULER_LARGE, sw.EULER_F64_FLAT),
    "euler_f32_flat_prec": (wl.EULER_PREC, sw.EULER_F32_FLAT),
    "euler_f64_flat_prec": (wl.EULER_PREC, sw.EULER_F64_FLAT),
    "ks_f64_prec": (wl.KS_PREC, sw.KS_F64),
}
# the default run: the 2^24-cell configuration in every equation id; the first
# leg is the headline value
DEFAULT_LEGS = ["heat_f64_prec", "heat_f32_prec", "euler_f64_prec", "euler_f32_prec",
                "euler_f64_flat_prec", "euler_f32_flat_prec", "ks_f64_prec"]

# algorithmic bytes of the swept working struct per cell (read + write per phase)
STRUCT_BYTES = {sw.HEAT_F64: 16, sw.HEAT_F32: 12, sw.EULER_F64: 56, sw.EULER_F32: 44,
                sw.EULER_F64_FLAT: 48, sw.EULER_F32_FLAT: 36, sw.KS_F64: 16}
# algorithmic HBM bytes per cell-update of the classic path
NAIVE_BYTES = {sw.HEAT_F64: 16, sw.HEAT_F32: 16, sw.EULER_F64: 200, sw.EULER_F32: 140,
               sw.EULER_F64_FLAT: 120, sw.EULER_F32_FLAT: 84, sw.KS_F64: 16}
# arithmetic operations per cell-update (one cell, one time step), counted from
# the scheme: every add, subtract, multiply, divide, square root, comparison and
# absolute value is one operation.  Heat: two differences, their sum, the
# multiply by r and the add (5); binary32 adds four Kahan operations.  Euler,
# per half step and cell: pressure 5, ratio 3, one face flux 64 (reciprocal
# ratio, two limiters, reconstruction, two primitive recoveries, two sound
# speeds, the two physical fluxes, the Rusanov dissipation), update 9;
# binary32 adds three Kahan operations per component in the corrector.
# Kuramoto-Sivashinsky: the second difference 3, the flux 2, the fourth
# difference 3, the update 7 (each stage once per cell).
OPS_PER_UPDATE = {sw.HEAT_F64: 5, sw.HEAT_F32: 8, sw.EULER_F64: 162, sw.EULER_F32: 171,
                  sw.EULER_F64_FLAT: 162, sw.EULER_F32_FLAT: 171, sw.KS_F64: 15}
# LDS bytes per heat cell-update of the register-blocked level sweep (read,
# write): every five levels a cell's two level slots (binary32: and its
# compensation) are read into registers and written back once
LDS_BYTES_PER_UPDATE = {sw.HEAT_F64: (16 / 5, 16 / 5), sw.HEAT_F32: (12 / 5, 12 / 5)}
PROFILES = os.path.join(ROOT, "profiles")
# the persistent launch of a heat-only batch (its kernel compiles only the heat body)
PERSISTENT_SOURCES = ["batch.hip", "batch.h", "tile_heat.h", "geom.h", "tile_job.h", "lanes.h",
                      "kernels.h"]
KERNEL_SOURCES = {
    sw.HEAT_F64: ["tile_heat.h", "heat.hip", "geom.h", "tile_job.h", "lanes.h", "kernels.h"],
    sw.HEAT_F32: ["tile_heat.h", "heat.hip", "geom.h", "tile_job.h", "lanes.h", "kernels.h"],
    sw.EULER_F64: ["tile_euler.h", "euler.hip", "geom.h", "tile_job.h", "lanes.h", "rn_ops.h"],
    sw.EULER_F32: ["tile_euler.h", "euler.hip", "geom.h", "tile_job.h", "lanes.h", "rn_ops.h"],
    sw.EULER_F64_FLAT: ["tile_flat.h", "tile_euler.h", "euler_flat.hip", "geom.h", "tile_job.h",
                        "lanes.h", "rn_ops.h"],
    sw.EULER_F32_FLAT: ["tile_flat.h", "tile_euler.h", "euler_flat.hip", "geom.h", "tile_job.h",
                        "lanes.h", "rn_ops.h"],
    sw.KS_F64: ["tile_ks.h", "ks.hip", "geom.h", "tile_job.h", "kernels.h"],
}


def kernel_source_hash(eq, schedule="phases") -> str:
    """sha256 of the sources of the swept kernel of `eq` under `schedule`."""
    import hashlib
    h = hashlib.sha256()
    for name in (PERSISTENT_SOURCES if schedule == "persistent" else KERNEL_SOURCES[eq]):
        with open(os.path.join(ROOT, "paper_1811_08282_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def leg_label(work, eq) -> str:
    """Name of a workload run in one equation id: <eq>_<precision>_n<N>_s<steps>."""
    layout = "_flattened" if eq in (sw.EULER_F64_FLAT, sw.EULER_F32_FLAT) else ""
    prec = "f64" if sw.is_f64(eq) else "f32"
    return f"{work.eq}_{prec}_n{work.n}_s{work.steps}{layout}"


def measured_counters(work, eq, width, threads, schedule="phases"):
    """Per-launch hardware counters of the swept kernel taken with rocprofv3 on
    this workload (profiles/<label>_phase_counters.txt for the phase
    launches, <label>_persistent_counters.txt for the persistent launch),
    or None when absent or taken on other kernel sources or another launch
    (width, workgroup size)."""
    kind = "persistent" if schedule == "persistent" else "phase"
    path = os.path.join(PROFILES, f"{leg_label(work, eq)}_{kind}_counters.txt")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if (rec.get("source_sha256") != kernel_source_hash(eq, schedule) or rec.get("width") != width
            or rec.get("threads") != threads):
        return None
    return rec


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pack_state(eq, q):
    q = np.asarray(q, np.float64)
    if eq in (sw.HEAT_F64, sw.KS_F64):
        return q.reshape(1, -1)
    if eq == sw.HEAT_F32:
        return np.stack([q.astype(np.float32), np.zeros(q.shape, np.float32)])
    if eq in (sw.EULER_F64, sw.EULER_F64_FLAT):
        return q
    return np.concatenate([q.astype(np.float32), np.zeros(q.shape, np.float32)])


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = float(np.max(np.abs(b)))
    err = float(np.max(np.abs(a - b)))
    return err / den if den else err


def _heat_windows(u0, steps, r, starts, span, fn):
    """Oracle values of cells [s, s + span) after `steps` steps, from a window
    wide enough that its own periodic wrap cannot reach its centre."""
    n = u0.shape[-1]
    out = []
    for s0 in starts:
        idx = np.arange(s0 - steps - 1, s0 + span + steps + 1) % n
        out.append((s0, fn(u0[..., idx], steps, r)))
    return out


_ORACLE_RESULTS = {}


def _oracle_cached(key, compute):
    """One oracle run per (workload, kind) per process: the two Euler layouts
    compute the same arithmetic and are checked against the same result."""
    if key not in _ORACLE_RESULTS:
        _ORACLE_RESULTS[key] = compute()
    return _ORACLE_RESULTS[key]


def verify_sample(work, eq, gpu):
    """Sampled comparison of one full-size GPU solve with the oracle.

    Heat: four dependency-cone windows of 16 cells each, stepped exactly.
    Euler on the Sod tiling: the solution is periodic with the tile, so one
    tile stepped by the oracle is every tile's exact value.  Same-precision
    comparisons must be bit-exact; binary32 runs also state their error
    against the binary64 oracle started from the binary32-rounded input.
    """
    import oracle
    q0 = wl.initial_state(work)
    out = {"reference": "oracle"}
    cached = _oracle_cached
    if eq == sw.KS_F64:
        span, reach = 16, 2 * work.steps + 2
        starts = [0, work.n // 3 + 5, work.n - 7, 12345 % work.n]
        ref = cached((work.name, "ks"), lambda: [
            oracle.ks_f64(q0[np.arange(s0 - reach, s0 + span + reach) % work.n], work.steps,
                          work.dt, work.dx)[reach: reach + span] for s0 in starts])
        got = np.concatenate([gpu[0][np.arange(s0, s0 + span) % work.n] for s0 in starts])
        want = np.concatenate(ref)
        out["bit_exact"] = bool(np.array_equal(got, want))
        out["max_abs_diff"] = float(np.max(np.abs(got - want)))
        out["sample"] = f"{len(starts)} windows of {span} cells (exact dependency cones, radius 2)"
        return out
    if eq in (sw.HEAT_F64, sw.HEAT_F32):
        r = work.dt / (work.dx * work.dx)
        span = 16
        starts = [0, work.n // 3 + 5, work.n - 7, 12345 % work.n]
        cells = lambda s0: np.arange(s0, s0 + span) % work.n  # noqa: E731
        sl = slice(work.steps + 1, work.steps + 1 + span)
        if eq == sw.HEAT_F64:
            ref = cached((work.name, "heat_f64"),
                         lambda: _heat_windows(q0, work.steps, r, starts, span, oracle.heat_f64))
            got = np.concatenate([gpu[0][cells(s0)] for s0, _ in ref])
            want = np.concatenate([v[sl] for _, v in ref])
            out["bit_exact"] = bool(np.array_equal(got, want))
        else:
            u32 = q0.astype(np.float32)
            pair = np.stack([u32, np.zeros_like(u32)])
            ref = cached((work.name, "heat_f32"), lambda: _heat_windows(
                pair, work.steps, r, starts, span,
                lambda w, k, a: np.stack(oracle.heat_f32(w[0], w[1], k, a))))
            got = np.concatenate([gpu[:, cells(s0)] for s0, _ in ref], axis=1)
            want = np.concatenate([v[:, sl] for _, v in ref], axis=1)
            out["bit_exact"] = bool(np.array_equal(got, want))
            ref64 = cached((work.name, "heat_f64_from_f32"), lambda: _heat_windows(
                u32.astype(np.float64), work.steps, r, starts, span, oracle.heat_f64))
            want64 = np.concatenate([v[sl] for _, v in ref64])
            out["rel_inf_vs_binary64"] = _rel(got[0], want64)
        out["max_abs_diff"] = float(np.max(np.abs(np.asarray(got, np.float64)
                                                  - np.asarray(want, np.float64))))
        out["sample"] = f"{len(starts)} windows of {span} cells (exact dependency cones)"
        return out
    lam = work.dt / work.dx
    tile = q0[:, : work.tile]
    tiles = work.n // work.tile
    if sw.is_f64(eq):
        want = cached((work.name, "euler_f64"), lambda: oracle.euler_f64(tile, work.steps, lam))
        got = gpu.reshape(3, tiles, work.tile)
        out["bit_exact"] = bool(np.array_equal(got, np.broadcast_to(want[:, None, :], got.shape)))
        out["max_abs_diff"] = float(np.max(np.abs(got - want[:, None, :])))
    else:
        t32 = tile.astype(np.float32)
        want_q, want_c = cached((work.name, "euler_f32"), lambda: oracle.euler_f32(
            t32, np.zeros_like(t32), work.steps, lam))
        want = np.concatenate([want_q, want_c])
        got = gpu.reshape(6, tiles, work.tile)
        out["bit_exact"] = bool(np.array_equal(got, np.broadcast_to(want[:, None, :], got.shape)))
        out["max_abs_diff"] = float(np.max(np.abs(got.astype(np.float64) - want[:, None, :])))
        ref64 = cached((work.name, "euler_f64_from_f32"), lambda: oracle.euler_f64(
            t32.astype(np.float64), work.steps, lam))
        g0 = got[:3, 0, :].astype(np.float64)
        out["rel_inf_vs_binary64"] = {k: _rel(g0[i], ref64[i]) for i, k in enumerate("rho m E".split())}
        out["rel_1_vs_binary64"] = {
            k: float(np.sum(np.abs(g0[i] - ref64[i])) / np.sum(np.abs(ref64[i])))
            for i, k in enumerate("rho m E".split())}
    out["sample"] = f"all {tiles} Sod tiles against one oracle tile ({work.tile} cells, {work.steps} steps)"
    return out


def cpu_baseline(work, eq, budget_s):
    """The oracle as it stands on the host cores, on a bounded sample of the
    workload (whole time steps of the whole grid until the budget is spent)."""
    import oracle
    q = wl.initial_state(work)
    chunk = 20
    done, t_used = 0, 0.0
    if eq == sw.KS_F64:
        arg = None
        cells = work.n

        def run(s, k, a):
            return oracle.ks_f64(s, k, work.dt, work.dx)
    elif eq in (sw.HEAT_F64, sw.HEAT_F32):
        arg = work.dt / (work.dx * work.dx)
        cells = work.n
        if eq == sw.HEAT_F64:
            run = oracle.heat_f64
        else:
            q = (q.astype(np.float32), np.zeros(q.shape, np.float32))

            def run(s, k, a):
                return oracle.heat_f32(s[0], s[1], k, a)
    else:
        # one Sod tile: the tiled problem is periodic with the tile's period
        q = q[:, : work.tile]
        arg = work.dt / work.dx
        cells = work.tile
        if sw.is_f64(eq):
            run = oracle.euler_f64
        else:
            q = (q.astype(np.float32), np.zeros(q.shape, np.float32))

            def run(s, k, a):
                return oracle.euler_f32(s[0], s[1], k, a)
    while t_used < budget_s and done < work.steps:
        t0 = time.perf_counter()
        q = run(q, chunk, arg)
        t_used += time.perf_counter() - t0
        done += chunk
    work_units = cells * done
    if work.eq == "euler" and done >= work.steps and t_used < budget_s:
        # one tile finished inside the budget: step a block of further whole
        # tiles (still periodic with the tile) over all steps, once
        more = min(int((budget_s - t_used) / t_used), work.n // work.tile - 1)
        if more > 0:
            block = wl.initial_state(work)[:, : more * work.tile]
            if not sw.is_f64(eq):
                block = (block.astype(np.float32), np.zeros(block.shape, np.float32))
            t0 = time.perf_counter()
            run(block, work.steps, arg)
            t_used += time.perf_counter() - t0
            work_units += more * work.tile * work.steps
            cells = (more + 1) * work.tile
    out = {
        "value": work_units / t_used,
        "unit": "cell-updates/s",
        "cores": oracle.threads_used(),
        "kind": "oracle",
        "sample": f"{cells} cells x {done} time steps of the same workload, "
                  f"{'binary64' if sw.is_f64(eq) else 'binary32 + Kahan'}, "
                  f"{t_used:.3g} s wall on {oracle.threads_used()} OpenMP threads ({cpu_model()})",
    }
    if work.name == wl.HEAT_SMALL.name and eq == sw.HEAT_F64:
        # the small configuration also on one host thread, whole workload
        t0 = time.perf_counter()
        oracle.heat_f64(wl.initial_state(work), work.steps, arg, threads=1)
        t1 = time.perf_counter() - t0
        out["single_thread"] = {"value": work.n * work.steps / t1, "unit": "cell-updates/s",
                                "cores": 1,
                                "sample": f"the whole workload, {work.n} cells x {work.steps} "
                                          f"time steps, {t1 * 1e3:.1f} ms"}
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


# ---- timing --------------------------------------------------------------------

def _problem(eq, dev, work, width):
    return dict(eq=eq, width=width, n_cells=work.n, n_steps=work.steps, dt=work.dt, dx=work.dx,
                d_state=dev.data_ptr())


def time_solves(torch, eq, state0, work, method, schedule, width, threads, reps, warmup,
                warmup_steps=None):
    """Time `reps` solves of the workload, each from the initial state
    restored by a device copy outside the timed region (HIP events on the
    launch stream, which is torch's current stream).  Returns the median ms,
    every ms, the device tensor holding the last solve's final state, and the
    width used."""
    import statistics
    pristine = torch.from_numpy(np.ascontiguousarray(state0)).cuda()
    dev = pristine.clone()
    stream = torch.cuda.current_stream()
    handle = stream.cuda_stream
    batch = None
    if method == "swept" and schedule == "persistent":
        torch.cuda.synchronize()
        batch = sw.Batch([_problem(eq, dev, work, width)], threads=threads)
        width = batch.width(0)

        def run(steps=None):
            batch.run(handle)
    else:
        def run(steps=None):
            sw.solve(eq, dev, work.steps if steps is None else steps, work.dt, work.dx,
                     method=method, width=width, threads=threads)
    for _ in range(warmup):
        dev.copy_(pristine)
        run(warmup_steps)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        dev.copy_(pristine)
        start.record(stream)
        run()
        stop.record(stream)
        stop.synchronize()
        times.append(start.elapsed_time(stop))
    if batch is not None:
        if batch.wait(handle) != sw.SW_OK:
            raise RuntimeError(sw.last_error())
        batch.close()
    torch.cuda.synchronize()
    del pristine
    return statistics.median(times), times, dev, width


def paper_style_ms(torch, eq, state0, work, method, schedule, width, threads):
    """One solve timed the way the paper times (Sec. 5): device allocation,
    the host-to-device copy of the state, the solve and the copy back."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev = torch.from_numpy(np.ascontiguousarray(state0)).cuda()
    if schedule == "persistent":
        handle = torch.cuda.current_stream().cuda_stream
        b = sw.Batch([_problem(eq, dev, work, width)], threads=threads)
        b.run(handle)
        if b.wait(handle) != sw.SW_OK:
            raise RuntimeError(sw.last_error())
        b.close()
    else:
        sw.solve(eq, dev, work.steps, work.dt, work.dx, method=method, width=width,
                 threads=threads)
    dev.cpu()
    return (time.perf_counter() - t0) * 1e3


# ---- rooflines -------------------------------------------------------------------

def rooflines(work, eq, schedule, width, threads, ms, rate):
    """Fractions of every unit that could bind the swept kernel, from the
    algorithmic counts and, where a counter record of the exact kernel
    sources and launch is committed under profiles/, from the counters.
    The binding unit is the one nearest its ceiling."""
    rad = sw.radius(eq)
    phases = sw.sw_phase_count(work.steps * sw.substeps(eq), width, rad)
    launches = 1 if schedule == "persistent" else phases
    launch_ms = ms / launches
    updates_per_launch = work.n * work.steps / launches
    tiles = work.n // width
    alg_bytes = (phases // launches) * tiles * ((width + 2 * rad) + width) * STRUCT_BYTES[eq]
    hbm_gbs = alg_bytes / (launch_ms * 1e-3) / 1e9
    units = {}
    units["hbm"] = {"achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": hbm_gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": alg_bytes}
    f64 = sw.is_f64(eq)
    ops = OPS_PER_UPDATE[eq]
    peak_alu = VECTOR_PEAK_TFLOPS[f64]
    units["alu"] = {"achieved": rate * ops / 1e12, "peak": peak_alu, "unit": "TFLOP/s",
                    "frac": rate * ops / 1e12 / peak_alu, "flops_per_cell_update": ops,
                    "precision": "binary64" if f64 else "binary32"}
    counters = measured_counters(work, eq, width, threads, schedule)
    rd = wr = None
    source = None
    if counters and counters.get("lds_load_bytes_per_launch") is not None:
        rd = counters["lds_load_bytes_per_launch"] / updates_per_launch
        wr = counters["lds_store_bytes_per_launch"] / updates_per_launch
        source = "counters"
    elif eq in LDS_BYTES_PER_UPDATE:
        rd, wr = LDS_BYTES_PER_UPDATE[eq]
        source = "algorithmic"
    if rd is not None:
        # seconds of port time per second: reads and writes one at a time,
        # each at its measured best rate
        busy = rate * (rd / (LDS_READ_B_PER_CLK * CUS * CLOCK_HZ)
                       + wr / (LDS_WRITE_B_PER_CLK * CUS * CLOCK_HZ))
        achieved = rate * (rd + wr) / 1e9
        units["lds"] = {"achieved": achieved, "peak": achieved / busy, "unit": "GB/s",
                        "frac": busy, "read_bytes_per_cell_update": rd,
                        "write_bytes_per_cell_update": wr, "source": source,
                        "peak_model": f"reads at {LDS_READ_B_PER_CLK} B/clk/CU and writes at "
                                      f"{LDS_WRITE_B_PER_CLK} B/clk/CU (measured), in turn"}
    # how close each unit runs to its ceiling: the algorithmic fractions, and
    # for the ALU also the share of CU-cycles the counters find it busy (the
    # scheme's divisions and square roots cost the hardware ten to twenty
    # instructions each, so its operation count understates the ALU's load)
    closeness = {k: units[k]["frac"] for k in units}
    if counters and counters.get("valu_mix_lane_insts_per_cell_update"):
        # diagnostic, not a roofline: the instructions the compiler issues for
        # those operations (a correctly rounded division is about ten), as
        # measured; a binary64 reciprocal or reciprocal square root holds its
        # SIMD four times as long as an add (SQ_ACTIVE_INST_VALU exceeds
        # SQ_INSTS_VALU by three per such instruction in the counter records)
        mix = counters["valu_mix_lane_insts_per_cell_update"]
        total = counters["valu_lane_insts_per_cell_update"]
        n64 = sum(mix.get(k, 0.0) for k in ("add_f64", "mul_f64", "fma_f64", "trans_f64"))
        units["valu"] = {
            "lane_insts_per_cell_update": total, "binary64_lane_insts_per_cell_update": n64,
            "transcendental_binary64_lane_insts_per_cell_update": mix.get("trans_f64", 0.0),
            "issue_wave_insts_per_cu_cycle": counters.get("valu_issue_per_cu_cycle"),
            "active_per_cu_cycle": counters.get("valu_active_per_cu_cycle"),
            "source": "counters"}
        active = counters.get("valu_active_per_cu_cycle")
        if active is not None:
            # binary32 instructions issue at up to twice the binary64 rate
            closeness["alu"] = max(closeness["alu"], active / (1.0 if f64 else 2.0))
    # the binding unit: the one nearest its ceiling; its fraction is reported
    # from the algorithmic count
    bound = max(closeness, key=closeness.get)
    traffic = counters.get("hbm_bytes_per_launch") if counters else None
    kernel = ("persistent swept kernel (heat body alone)" if schedule == "persistent"
              else "swept phase kernel")
    out = {"bound": bound, "achieved": units[bound]["achieved"], "peak": units[bound]["peak"],
           "unit": units[bound]["unit"], "frac": units[bound]["frac"], "traffic": traffic,
           "closeness_to_ceiling": closeness,
           "kernel": kernel, "launch_ms": launch_ms, "launches_per_step": launches,
           "counters": "profiles/" + f"{leg_label(work, eq)}_"
                       f"{'persistent' if schedule == 'persistent' else 'phase'}_counters.txt"
                       if counters else None}
    out.update(units)
    return out


# ---- one leg: swept and classic on one workload in one equation id ---------------

def persistent_route(eq, n, width):
    """The rule swept_solve follows: a heat grid runs as one persistent
    launch when its tiles are 1792 cells wide or more and more than 1024 in
    number (measured on MI355X at 6000 steps, binary64, W = 2048: 2.94e12
    against 2.74e12 cell-updates/s at 2^22 cells, level at 2^21, 1.36e12
    against 1.73e12 at 2^20; 2048 tiles: 2.9e12 against 2.7e12 at W = 1792,
    level at W = 1280, 1.9e12 against 2.1e12 at W = 1024)."""
    return eq in (sw.HEAT_F64, sw.HEAT_F32) and width >= 1792 and n // width > 1024


def default_schedule(eq, work):
    # Euler and Kuramoto-Sivashinsky phases last 6-55 ms: the drain between
    # launches costs little, and for Euler the two are level or the phase
    # launches win
    width = sw.sw_default_width(eq, work.n)
    return "persistent" if persistent_route(eq, work.n, width) else "phases"


def run_leg(torch, work, eq, args, reps, naive_reps, warmup, verify=True):
    schedule = args.schedule if args.schedule != "auto" else default_schedule(eq, work)
    state0 = pack_state(eq, wl.initial_state(work))
    updates = work.n * work.steps
    if schedule == "persistent":
        width, threads = args.width, args.threads or 256
    else:
        width = args.width or sw.sw_default_width(eq, work.n)
        threads = args.threads or sw.sw_default_threads(eq, width)
    # a short warm-up solve is enough for the slow legs (it loads the code
    # and sizes the working arrays); the persistent launch always runs whole
    warm_steps = None if (schedule == "persistent" or work.eq == "heat") else min(work.steps, 100)
    label = leg_label(work, eq)
    log(f"[bench] {label}: swept ({schedule}), {reps} timed solves")
    ms, times, dev, width = time_solves(torch, eq, state0, work, "swept", schedule, width,
                                        threads, reps, warmup, warm_steps)
    phases = sw.sw_phase_count(work.steps * sw.substeps(eq), width, sw.radius(eq))
    rate = updates / (ms * 1e-3)
    log(f"[bench] {label}: swept {ms:.3f} ms/solve ({rate:.4g} cell-updates/s), W={width}, "
        f"threads={threads}, phases={phases}")
    final = dev.cpu().numpy()
    del dev
    leg = {"workload": label, "eq": eq, "precision": "binary64" if sw.is_f64(eq) else "binary32",
           "n_cells": work.n, "time_steps": work.steps, "width": width, "threads": threads,
           "schedule": schedule, "phases": phases,
           "swept": {"value": rate, "ms_per_solve": ms, "ms_all": times, "reps": reps}}
    if naive_reps:
        log(f"[bench] {label}: naive, {naive_reps} timed solves")
        nms, ntimes, ndev, _ = time_solves(torch, eq, state0, work, "naive", "phases", 0, 0,
                                           naive_reps, 1, 10)
        del ndev
        nrate = updates / (nms * 1e-3)
        log(f"[bench] {label}: naive {nms:.3f} ms/solve ({nrate:.4g} cell-updates/s)")
        leg["naive"] = {"value": nrate, "ms_per_solve": nms, "ms_all": ntimes, "reps": naive_reps,
                        "launches_per_solve": work.steps * sw.substeps(eq),
                        "hbm_roofline_value": HBM_PEAK_GBS * 1e9 / NAIVE_BYTES[eq]}
        leg["swept_over_naive"] = rate / nrate
    leg["effective_roofline_frac"] = rate / (HBM_PEAK_GBS * 1e9 / NAIVE_BYTES[eq])
    leg["roofline"] = rooflines(work, eq, schedule, width, threads, ms, rate)
    if verify:
        t0 = time.perf_counter()
        v = verify_sample(work, eq, final)
        v["seconds"] = time.perf_counter() - t0
        leg["error_vs_oracle"] = v
        log(f"[bench] {label}: oracle check bit_exact={v['bit_exact']}")
    return leg, state0


# ---- width sweep -----------------------------------------------------------------

def width_sweep(torch, work, eq, widths, reps, naive_reps):
    """Swept (phase launches and the persistent launch) at every width, and
    classic once, on one workload; every solve from the restored state."""
    state0 = pack_state(eq, wl.initial_state(work))
    updates = work.n * work.steps
    rows = []
    for w in widths:
        row = {"width": w}
        threads = sw.sw_default_threads(eq, w)
        ms, times, dev, _ = time_solves(torch, eq, state0, work, "swept", "phases", w, threads,
                                        reps, 1)
        del dev
        row["phases"] = {"value": updates / (ms * 1e-3), "ms_per_solve": ms, "threads": threads,
                         "launches": sw.sw_phase_count(work.steps * sw.substeps(eq), w,
                                                       sw.radius(eq))}
        if eq in (sw.HEAT_F64, sw.HEAT_F32) and w >= 64:
            pms, _, dev, _ = time_solves(torch, eq, state0, work, "swept", "persistent", w, 256,
                                         reps, 1)
            del dev
            row["persistent"] = {"value": updates / (pms * 1e-3), "ms_per_solve": pms,
                                 "threads": 256}
        log(f"[bench] sweep W={w}: {json.dumps(row)}")
        rows.append(row)
    nms, _, dev, _ = time_solves(torch, eq, state0, work, "naive", "phases", 0, 0, naive_reps, 1)
    del dev
    return {"workload": leg_label(work, eq), "reps": reps, "rows": rows,
            "naive": {"value": updates / (nms * 1e-3), "ms_per_solve": nms, "reps": naive_reps}}


# the paper's grid sizes (Sec. 5) among powers of two, and its 6000-step average
GRID_SIZES = [1 << 12, 1 << 14, 1 << 16, 1 << 18, 500000, 1000000, 1 << 20, 1 << 22, 5000000,
              10000000, 1 << 24]
GRID_STEPS = 6000


def grid_sweep(torch, eq, sizes, steps, reps):
    """swept_solve (library width, workgroup size and schedule) against the
    classic solve over grid sizes, with the state resident in HBM and the way
    the paper times (allocation and host copies included); every pair of
    final states compared bit for bit."""
    rows = []
    for n in sizes:
        if eq == sw.HEAT_F64:
            work = wl.Workload(f"heat_f64_n{n}_s{steps}", "heat", n, steps, 0.25, 1.0, 7)
        else:
            work = wl.Workload(f"euler_f64_n{n}_s{steps}", "euler", n, steps, 0.1, 1.0, None,
                               1 << 14)
        state0 = pack_state(eq, wl.initial_state(work))
        updates = n * steps
        width = sw.sw_default_width(eq, n)
        sms, _, sdev, _ = time_solves(torch, eq, state0, work, "swept", "phases", 0, 0, reps, 1)
        nms, _, ndev, _ = time_solves(torch, eq, state0, work, "naive", "phases", 0, 0, reps, 1)
        same = bool(torch.equal(sdev, ndev))
        del sdev, ndev
        sp = paper_style_ms(torch, eq, state0, work, "swept", "phases", 0, 0)
        npms = paper_style_ms(torch, eq, state0, work, "naive", "phases", 0, 0)
        row = {"n_cells": n, "width": width,
               "schedule": "persistent" if persistent_route(eq, n, width) else "phases",
               "swept": updates / (sms * 1e-3), "classic": updates / (nms * 1e-3),
               "swept_over_classic": nms / sms, "swept_equals_classic": same,
               "with_host_copies": {"swept_ms": sp, "classic_ms": npms,
                                    "swept_over_classic": npms / sp}}
        log(f"[bench] grid {leg_label(work, eq)}: {json.dumps(row)}")
        rows.append(row)
    return {"equation": "heat" if eq == sw.HEAT_F64 else "euler", "precision": "binary64",
            "time_steps": steps, "reps": reps, "rows": rows}


def wf_sweep(torch, work, eq, tiles_per_thread, host_threads, reps):
    """The swept solve shared with host threads (sw_opts.work_factor), against
    the GPU alone, on one workload; each host thread takes k tiles for k in
    tiles_per_thread (work factor T/k - P for T tiles, P threads)."""
    import statistics
    state0 = pack_state(eq, wl.initial_state(work))
    width = sw.sw_default_width(eq, work.n)
    tiles = work.n // width
    updates = work.n * work.steps
    pristine = torch.from_numpy(np.ascontiguousarray(state0)).cuda()
    dev = pristine.clone()

    def timed(wf):
        times = []
        for _ in range(reps + 1):
            dev.copy_(pristine)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sw.solve(eq, dev, work.steps, work.dt, work.dx, method="swept", width=width,
                     work_factor=wf, host_threads=host_threads if wf else 0)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        return statistics.median(times[1:])

    rows = []
    ms = timed(0)
    rows.append({"work_factor": 0, "host_tiles": 0, "gpu_tiles": tiles, "ms_per_solve": ms,
                 "value": updates / (ms * 1e-3)})
    log(f"[bench] wf sweep {leg_label(work, eq)}: GPU alone {ms:.1f} ms")
    for k in tiles_per_thread:
        wf = tiles // k - host_threads
        if wf < 1:
            continue
        kt = tiles // (wf + host_threads)
        ms = timed(wf)
        row = {"work_factor": wf, "tiles_per_host_thread": kt, "host_tiles": host_threads * kt,
               "gpu_tiles": tiles - host_threads * kt,
               "gpu_over_host_thread": (tiles - host_threads * kt) / kt,
               "ms_per_solve": ms, "value": updates / (ms * 1e-3)}
        log(f"[bench] wf sweep: {json.dumps(row)}")
        rows.append(row)
    return {"workload": leg_label(work, eq), "width": width, "tiles": tiles,
            "host_threads": host_threads, "reps": reps, "rows": rows}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5,
                    help="timed solves of the headline workload (median reported)")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves before the timed ones")
    ap.add_argument("--workload", default=None, choices=sorted(WORKLOADS),
                    help="measure one workload only (default: every leg at 2^24 cells)")
    ap.add_argument("--width", type=int, default=0, help="triangle width (0: library choice)")
    ap.add_argument("--threads", type=int, default=0,
                    help="workgroup size of the swept kernel (0: library choice)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "phases", "persistent"],
                    help="one launch per phase, or one persistent launch per solve "
                         "(auto: swept_solve's rule, persistent for heat grids of more than "
                         "1024 tiles of 1792 cells or more)")
    ap.add_argument("--naive-reps", type=int, default=3, help="timed classic solves of heat legs")
    ap.add_argument("--euler-reps", type=int, default=1,
                    help="timed swept and classic solves of each Euler leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-naive", action="store_true", help="skip the classic-path timing")
    ap.add_argument("--no-verify", action="store_true", help="skip the sampled oracle checks")
    ap.add_argument("--sweep", default=None, choices=["c2", "c1", "wf", "grid"],
                    help="width sweep of the 2^22-cell heat workload (c2, widths 64 to the LDS "
                         "limit), the 1024-cell one at W = 64 (c1), the GPU work factor of a "
                         "solve shared with host threads (wf: heat 2^22 cells, Euler 2^24), or "
                         "swept against classic over grid sizes 2^12 to 2^24 and the paper's "
                         "5e5 to 1e7 (grid: heat and Euler binary64, 6000 steps)")
    ap.add_argument("--host-threads", type=int, default=8,
                    help="host threads of the work-factor sweep")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the swept path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(args.steps, 1)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8}))
        return 0
    sw.load()

    if args.sweep == "grid":
        res = {"metric": "cell-updates/s",
               "sweeps": [grid_sweep(torch, sw.HEAT_F64, GRID_SIZES, GRID_STEPS, max(args.steps, 1)),
                          grid_sweep(torch, sw.EULER_F64, GRID_SIZES, GRID_STEPS, 1)]}
        print(json.dumps(res), flush=True)
        return 0
    if args.sweep == "wf":
        res = {"metric": "cell-updates/s",
               "sweeps": [wf_sweep(torch, wl.HEAT_LARGE, sw.HEAT_F64, [1, 2, 4], args.host_threads,
                                   max(args.steps, 1)),
                          wf_sweep(torch, wl.EULER_PREC, sw.EULER_F64, [1, 2, 4, 8],
                                   args.host_threads, 1)]}
        print(json.dumps(res), flush=True)
        return 0
    if args.sweep:
        if args.sweep == "c2":
            work, eq = wl.HEAT_LARGE, sw.HEAT_F64
            wmax = sw.sw_max_width(eq)
            widths = [w for w in (64, 128, 256, 512, 1024, 2048, 4096, 8192) if w <= wmax]
            res = width_sweep(torch, work, eq, widths, max(args.steps, 1), 1)
        else:
            work, eq = wl.HEAT_SMALL, sw.HEAT_F64
            res = width_sweep(torch, work, eq, [64], max(args.steps, 1), max(args.steps, 1))
        res["metric"] = "cell-updates/s"
        print(json.dumps(res), flush=True)
        return 0

    legs_spec = ([(args.workload,) + WORKLOADS[args.workload]] if args.workload else
                 [(name,) + WORKLOADS[name] for name in DEFAULT_LEGS])
    legs = []
    head_state0 = None
    for i, (name, work, eq) in enumerate(legs_spec):
        euler = work.eq == "euler"
        if i == 0:
            reps, warmup = args.steps, args.warmup
        else:
            reps, warmup = (args.euler_reps, 1) if euler else (min(args.steps, 5), 1)
        naive_reps = 0 if args.no_naive else (args.euler_reps if euler else args.naive_reps)
        leg, state0 = run_leg(torch, work, eq, args, reps, naive_reps, warmup,
                              verify=not args.no_verify)
        if i == 0:
            head_state0 = state0
        legs.append(leg)

    head = legs[0]
    name, work, eq = legs_spec[0]
    ms = head["swept"]["ms_per_solve"]
    value = head["swept"]["value"]
    paper_ms = paper_style_ms(torch, eq, head_state0, work, "swept", head["schedule"],
                              head["width"], head["threads"])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if sw.is_f64(eq) else "f32",
        "data": "synthetic",
        "config": {"workload": head["workload"], "n_cells": work.n, "time_steps": work.steps,
                   "width": head["width"], "threads": head["threads"],
                   "schedule": head["schedule"], "phases": head["phases"], "method": "swept",
                   "parallelism": "single-gpu",
                   "step": f"one solve: {work.steps} time steps of all {work.n} cells"},
        "naive": head.get("naive"),
        "swept_over_naive": head.get("swept_over_naive"),
        "effective_roofline_frac": head["effective_roofline_frac"],
        "roofline": head["roofline"],
        "error_vs_oracle": head.get("error_vs_oracle"),
        "with_host_copies": {"ms_per_step": paper_ms, "value": work.n * work.steps / (paper_ms * 1e-3),
                             "note": "one solve including device allocation and the host-to-device "
                                     "and device-to-host copies of the state (PCIe)"},
        "legs": [{k: v for k, v in leg.items() if k != "eq"} for leg in legs],
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(work, eq, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
