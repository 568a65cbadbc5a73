#!/usr/bin/env python3
"""Benchmark of the swept-rule hot path on one MI355X.

One benchmark step is one full solve of the workload through the C ABI:
every phase of the swept schedule -- Up Triangle, Diamonds, Down Triangle --
over the whole grid for all its time steps.  Two schedules of the same
phases exist: one kernel launch per phase (``swept_solve``), or one
persistent launch that overlaps consecutive phases tile by tile (the batched
launch with the single problem, ``sw_batch_run``).  By default the heat
workloads of 2^20 cells and more use the persistent launch and the others
the phase launches, the faster of the two for each on MI355X.  The default workload is
the 1D heat equation (FTCS, binary64) on 2^22 periodic cells, r = 1/4,
seeded random-mode initial condition, 20000 time steps.

Prints ONE JSON line: the swept throughput in cell-updates/s (value), the
classic one-launch-per-step throughput on the same workload, the roofline
of the dominant kernel (timed live with HIP events on the library's stream)
and the plain CPU oracle timed on a bounded sample of the same workload.
Inputs are resident in HBM before the timed region starts.
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
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6  # counts an FMA as two flops

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
}

# algorithmic bytes of the swept working struct per cell (read + write per phase)
STRUCT_BYTES = {sw.HEAT_F64: 16, sw.HEAT_F32: 12, sw.EULER_F64: 56, sw.EULER_F32: 44,
                sw.EULER_F64_FLAT: 48, sw.EULER_F32_FLAT: 36}
# algorithmic HBM bytes per cell-update of the classic path
NAIVE_BYTES = {sw.HEAT_F64: 16, sw.HEAT_F32: 16, sw.EULER_F64: 200, sw.EULER_F32: 140,
               sw.EULER_F64_FLAT: 120, sw.EULER_F32_FLAT: 84}
# arithmetic operations per cell-update (one cell, one time step), counted from
# the scheme: every add, subtract, multiply, divide, square root, comparison and
# absolute value is one operation.  Heat: two differences, their sum, the
# multiply by r and the add (5); binary32 adds four Kahan operations.  Euler,
# per half step and cell: pressure 5, ratio 3, one face flux 64 (reciprocal
# ratio, two limiters, reconstruction, two primitive recoveries, two sound
# speeds, the two physical fluxes, the Rusanov dissipation), update 9;
# binary32 adds three Kahan operations per component in the corrector.
OPS_PER_UPDATE = {sw.HEAT_F64: 5, sw.HEAT_F32: 8, sw.EULER_F64: 162, sw.EULER_F32: 171,
                  sw.EULER_F64_FLAT: 162, sw.EULER_F32_FLAT: 171}
# vector lane-operation issue rate with no fused or packed forms (the kernels
# use neither): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# LDS port: 128 bytes per clock per CU
LDS_PEAK_GBS = 256 * 128 * 2.4e9 / 1e9
# LDS bytes per heat cell-update of the level sweep: three neighbour reads and
# one write (binary32: plus the compensation read and write)
LDS_BYTES_PER_UPDATE = {sw.HEAT_F64: 32, sw.HEAT_F32: 24}
PROFILES = os.path.join(ROOT, "profiles")
# the persistent launch of a heat-only batch (its kernel compiles only the heat body)
PERSISTENT_SOURCES = ["batch.hip", "batch.h", "tile_heat.h", "geom.h", "tile_job.h"]
KERNEL_SOURCES = {
    sw.HEAT_F64: ["tile_heat.h", "heat.hip", "geom.h", "tile_job.h"],
    sw.HEAT_F32: ["tile_heat.h", "heat.hip", "geom.h", "tile_job.h"],
    sw.EULER_F64: ["tile_euler.h", "euler.hip", "geom.h", "tile_job.h"],
    sw.EULER_F32: ["tile_euler.h", "euler.hip", "geom.h", "tile_job.h"],
    sw.EULER_F64_FLAT: ["tile_flat.h", "tile_euler.h", "euler_flat.hip", "geom.h", "tile_job.h"],
    sw.EULER_F32_FLAT: ["tile_flat.h", "tile_euler.h", "euler_flat.hip", "geom.h", "tile_job.h"],
}


def kernel_source_hash(eq, schedule="phases") -> str:
    """sha256 of the sources of the swept kernel of `eq` under `schedule`."""
    import hashlib
    h = hashlib.sha256()
    for name in (PERSISTENT_SOURCES if schedule == "persistent" else KERNEL_SOURCES[eq]):
        with open(os.path.join(ROOT, "paper_1811_08282_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_counters(work, eq, width, threads, schedule="phases"):
    """Per-launch hardware counters of the swept kernel taken with rocprofv3 on
    this workload (profiles/<workload>_phase_counters.txt for the phase
    launches, <workload>_persistent_counters.txt for the persistent launch),
    or None when absent or taken on other kernel sources or another launch
    (width, workgroup size)."""
    layout = "_flattened" if eq in (sw.EULER_F64_FLAT, sw.EULER_F32_FLAT) else ""
    kind = "persistent" if schedule == "persistent" else "phase"
    path = os.path.join(PROFILES, f"{work.name}{layout}_{kind}_counters.txt")
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
    if eq == sw.HEAT_F64:
        return q.reshape(1, -1)
    if eq == sw.HEAT_F32:
        return np.stack([q.astype(np.float32), np.zeros(q.shape, np.float32)])
    if eq in (sw.EULER_F64, sw.EULER_F64_FLAT):
        return q
    return np.concatenate([q.astype(np.float32), np.zeros(q.shape, np.float32)])


def time_solves(torch, eq, state0, work, method, width, reps, warmup, threads=0):
    """Mean ms per solve over `reps` solves (events on the library's stream)."""
    dev = torch.from_numpy(np.ascontiguousarray(state0)).cuda()
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        sw.solve(eq, dev, work.steps, work.dt, work.dx, method=method, width=width,
                 threads=threads)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    t0 = time.perf_counter()
    for _ in range(reps):
        sw.solve(eq, dev, work.steps, work.dt, work.dx, method=method, width=width,
                 threads=threads)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return start.elapsed_time(stop) / reps, wall / reps


def _batch_problem(eq, dev, work, width):
    return dict(eq=eq, width=width, n_cells=work.n, n_steps=work.steps, dt=work.dt, dx=work.dx,
                d_state=dev.data_ptr())


def time_persistent(torch, eq, state0, work, width, threads, reps, warmup):
    """Mean ms per solve over `reps` persistent launches of the batch holding
    the single problem (events on torch's current stream, the launch stream);
    also returns the width the batch chose."""
    dev = torch.from_numpy(np.ascontiguousarray(state0)).cuda()
    torch.cuda.synchronize()
    b = sw.Batch([_batch_problem(eq, dev, work, width)], threads=threads)
    stream = torch.cuda.current_stream()
    handle = stream.cuda_stream
    for _ in range(warmup):
        b.run(handle)
    if b.wait(handle) != sw.SW_OK:
        raise RuntimeError(sw.last_error())
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    t0 = time.perf_counter()
    for _ in range(reps):
        b.run(handle)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    if b.wait(handle) != sw.SW_OK:
        raise RuntimeError(sw.last_error())
    chosen = b.width(0)
    b.close()
    return start.elapsed_time(stop) / reps, wall / reps, chosen


def solve_once(torch, eq, state0, work, width, threads, schedule):
    """One solve from state0 on the given schedule; returns the device tensor."""
    dev = torch.from_numpy(np.ascontiguousarray(state0)).cuda()
    if schedule == "persistent":
        torch.cuda.synchronize()
        b = sw.Batch([_batch_problem(eq, dev, work, width)], threads=threads)
        handle = torch.cuda.current_stream().cuda_stream
        b.run(handle)
        if b.wait(handle) != sw.SW_OK:
            raise RuntimeError(sw.last_error())
        b.close()
    else:
        sw.solve(eq, dev, work.steps, work.dt, work.dx, method="swept", width=width,
                 threads=threads)
    return dev


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
    if eq in (sw.HEAT_F64, sw.HEAT_F32):
        r = work.dt / (work.dx * work.dx)
        span = 16
        starts = [0, work.n // 3 + 5, work.n - 7, 12345 % work.n]
        cells = lambda s0: np.arange(s0, s0 + span) % work.n  # noqa: E731
        sl = slice(work.steps + 1, work.steps + 1 + span)
        if eq == sw.HEAT_F64:
            ref = _heat_windows(q0, work.steps, r, starts, span, oracle.heat_f64)
            got = np.concatenate([gpu[0][cells(s0)] for s0, _ in ref])
            want = np.concatenate([v[sl] for _, v in ref])
            out["bit_exact"] = bool(np.array_equal(got, want))
        else:
            u32 = q0.astype(np.float32)
            pair = np.stack([u32, np.zeros_like(u32)])
            ref = _heat_windows(pair, work.steps, r, starts, span,
                                lambda w, k, a: np.stack(oracle.heat_f32(w[0], w[1], k, a)))
            got = np.concatenate([gpu[:, cells(s0)] for s0, _ in ref], axis=1)
            want = np.concatenate([v[:, sl] for _, v in ref], axis=1)
            out["bit_exact"] = bool(np.array_equal(got, want))
            ref64 = _heat_windows(u32.astype(np.float64), work.steps, r, starts, span,
                                  oracle.heat_f64)
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
        want = oracle.euler_f64(tile, work.steps, lam)
        got = gpu.reshape(3, tiles, work.tile)
        out["bit_exact"] = bool(np.array_equal(got, np.broadcast_to(want[:, None, :], got.shape)))
        out["max_abs_diff"] = float(np.max(np.abs(got - want[:, None, :])))
    else:
        t32 = tile.astype(np.float32)
        want_q, want_c = oracle.euler_f32(t32, np.zeros_like(t32), work.steps, lam)
        want = np.concatenate([want_q, want_c])
        got = gpu.reshape(6, tiles, work.tile)
        out["bit_exact"] = bool(np.array_equal(got, np.broadcast_to(want[:, None, :], got.shape)))
        out["max_abs_diff"] = float(np.max(np.abs(got.astype(np.float64) - want[:, None, :])))
        ref64 = oracle.euler_f64(t32.astype(np.float64), work.steps, lam)
        g0 = got[:3, 0, :].astype(np.float64)
        out["rel_inf_vs_binary64"] = {k: _rel(g0[i], ref64[i]) for i, k in enumerate("rho m E".split())}
        out["rel_1_vs_binary64"] = {
            k: float(np.sum(np.abs(g0[i] - ref64[i])) / np.sum(np.abs(ref64[i])))
            for i, k in enumerate("rho m E".split())}
    out["sample"] = f"all {tiles} Sod tiles against one oracle tile ({work.tile} cells, {work.steps} steps)"
    return out


def cpu_baseline(work, eq, budget_s, gpu_final=None):
    """The oracle as it stands on the host cores, on a bounded sample of the
    workload; with `gpu_final` (one full-size GPU solve from the same input)
    the same leg also checks that solve against the oracle on a sample."""
    import oracle
    q = wl.initial_state(work)
    chunk = 20
    done, t_used = 0, 0.0
    if eq in (sw.HEAT_F64, sw.HEAT_F32):
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
    if eq not in (sw.HEAT_F64, sw.HEAT_F32) and done >= work.steps and t_used < budget_s:
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
    if gpu_final is not None:
        t0 = time.perf_counter()
        out["verify"] = verify_sample(work, eq, gpu_final)
        out["verify"]["seconds"] = time.perf_counter() - t0
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


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed solves")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves")
    ap.add_argument("--workload", default="heat_f64_large", choices=sorted(WORKLOADS))
    ap.add_argument("--width", type=int, default=0, help="triangle width (0: library choice)")
    ap.add_argument("--threads", type=int, default=0,
                    help="workgroup size of the swept kernel (0: library choice)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "phases", "persistent"],
                    help="one launch per phase, or one persistent launch per solve "
                         "(auto: persistent for heat grids of 2^20 cells and more)")
    ap.add_argument("--naive-reps", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-naive", action="store_true", help="skip the classic-path timing")
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
    work, eq = WORKLOADS[args.workload]
    sw.load()
    schedule = args.schedule
    if schedule == "auto":
        # measured on MI355X: the persistent launch wins for heat grids of
        # 2^20 cells and more (2^22: 2.12e12 against 1.98e12); on a grid of
        # a few tiles (1024 cells) the phase launches are slightly faster, and
        # for Euler the two are level or the phase launches win
        big_heat = eq in (sw.HEAT_F64, sw.HEAT_F32) and work.n >= (1 << 20)
        schedule = "persistent" if big_heat else "phases"
    state0 = pack_state(eq, wl.initial_state(work))
    updates = work.n * work.steps
    if schedule == "persistent":
        threads = args.threads or 256
        ms, wall_ms, width = time_persistent(torch, eq, state0, work, args.width, threads,
                                             args.steps, args.warmup)
    else:
        width = args.width or sw.sw_default_width(eq, work.n)
        threads = args.threads or sw.sw_default_threads(eq, width)
    final_level = work.steps * sw.substeps(eq)
    phases = sw.sw_phase_count(final_level, width, sw.radius(eq))
    log(f"[bench] workload {work.name} eq={eq} W={width} threads={threads} phases={phases} "
        f"schedule={schedule}")
    if schedule == "phases":
        ms, wall_ms = time_solves(torch, eq, state0, work, "swept", width, args.steps,
                                  args.warmup, threads)
    log(f"[bench] swept {ms:.3f} ms/solve ({updates / ms * 1e3:.4g} cell-updates/s)")
    phase_launches = None
    if schedule == "persistent":
        # the same solve through swept_solve (one launch per phase), for reference
        pw = sw.sw_default_width(eq, work.n)
        pt = sw.sw_default_threads(eq, pw)
        pms, _ = time_solves(torch, eq, state0, work, "swept", pw, args.steps, args.warmup, pt)
        phase_launches = {"value": updates / (pms * 1e-3), "ms_per_step": pms, "width": pw,
                          "threads": pt, "launches_per_step": sw.sw_phase_count(
                              work.steps * sw.substeps(eq), pw, sw.radius(eq))}
        log(f"[bench] swept, one launch per phase {pms:.3f} ms/solve "
            f"({updates / pms * 1e3:.4g} cell-updates/s)")
    naive_ms = float("nan")
    if not args.no_naive:
        naive_ms, _ = time_solves(torch, eq, state0, work, "naive", 0, args.naive_reps, 1)
        log(f"[bench] naive {naive_ms:.3f} ms/solve ({updates / naive_ms * 1e3:.4g} cell-updates/s)")

    # the paper's timing protocol also counts device allocation and the copies
    # to and from the host; reported beside the HBM-resident figure only
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev = solve_once(torch, eq, state0, work, width, threads, schedule)
    host_final = dev.cpu().numpy()
    paper_ms = (time.perf_counter() - t0) * 1e3
    del dev, host_final

    value = updates / (ms * 1e-3)
    naive_value = updates / (naive_ms * 1e-3) if naive_ms == naive_ms else None
    # dominant kernel: the swept phase kernel (one launch per phase) or the
    # persistent kernel (one launch per solve, every phase inside)
    launches = 1 if schedule == "persistent" else phases
    launch_ms = ms / launches
    tiles = work.n // width
    alg_bytes = (phases // launches) * tiles * ((width + 2 * sw.radius(eq)) + width) \
        * STRUCT_BYTES[eq]
    achieved_gbs = alg_bytes / (launch_ms * 1e-3) / 1e9
    hbm = {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved_gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": alg_bytes}
    counters = measured_counters(work, eq, width, threads, schedule)
    traffic = counters.get("hbm_bytes_per_launch") if counters else None
    ops = OPS_PER_UPDATE[eq]
    achieved = value * ops / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS,
                "unit": "TFLOP/s", "frac": achieved / ALU_PEAK_TOPS, "traffic": traffic,
                "ops_per_cell_update": ops, "flops_per_launch": updates * ops / launches,
                "kernel": ("persistent swept kernel (heat body alone)" if schedule == "persistent"
                           else "swept phase kernel"),
                "launch_ms": launch_ms, "launches_per_step": launches, "hbm": hbm}
    if eq in LDS_BYTES_PER_UPDATE:
        lds_gbs = value * LDS_BYTES_PER_UPDATE[eq] / 1e9
        roofline["lds"] = {"achieved": lds_gbs, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                           "frac": lds_gbs / LDS_PEAK_GBS,
                           "bytes_per_cell_update": LDS_BYTES_PER_UPDATE[eq]}
    if counters and counters.get("lds_load_bytes_per_launch") is not None:
        # LDS bytes the SQ counters saw (64-byte units of the load and store
        # bandwidth counters), per cell-update and per second of launch time
        lds_bytes = counters["lds_load_bytes_per_launch"] + counters["lds_store_bytes_per_launch"]
        measured = {"bytes_per_cell_update": lds_bytes / (updates / launches),
                    "achieved": lds_bytes / (launch_ms * 1e-3) / 1e9, "peak": LDS_PEAK_GBS,
                    "unit": "GB/s"}
        measured["frac"] = measured["achieved"] / LDS_PEAK_GBS
        roofline.setdefault("lds", {})["measured"] = measured
    # the unit that binds the kernel, from the counter profile and the LDS
    # probe: the heat level sweep saturates the LDS port (its measured
    # pattern ceiling is 3.39 updates per clock per CU), the Euler kernels
    # the VALU issue (correctly rounded divisions and square roots)
    roofline["binding_unit"] = "lds" if eq in LDS_BYTES_PER_UPDATE else "valu"
    if counters and counters.get("valu_insts_per_launch"):
        # wave-level VALU instructions issued per second over the chip's issue
        # rate (one wave instruction per clock per CU)
        rate = counters["valu_insts_per_launch"] / (launch_ms * 1e-3)
        roofline["valu_issue"] = {
            "insts_per_cell_update": counters["valu_insts_per_launch"] * 64 / (updates / launches),
            "achieved": rate / 1e9, "peak": 256 * 2.4, "unit": "G wave-insts/s",
            "frac": rate / (256 * 2.4e9)}
    # with a counter profile, the unit nearer its ceiling binds (binary32 heat
    # issues VALU instructions at 94 % of the chip's rate while its LDS port
    # runs at 73 %)
    lds_meas = roofline.get("lds", {}).get("measured")
    if "valu_issue" in roofline and lds_meas:
        roofline["binding_unit"] = ("valu" if roofline["valu_issue"]["frac"] > lds_meas["frac"]
                                    else "lds")
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
        "config": {"workload": work.name + ("_flattened" if eq in (sw.EULER_F64_FLAT, sw.EULER_F32_FLAT) else ""),
                   "n_cells": work.n, "time_steps": work.steps, "width": width,
                   "threads": threads, "schedule": schedule, "phases": phases,
                   "method": "swept", "parallelism": "single-gpu"},
        "swept_phase_launches": phase_launches,
        "naive": {"value": naive_value, "ms_per_step": naive_ms,
                  "hbm_roofline_value": HBM_PEAK_GBS * 1e9 / NAIVE_BYTES[eq]},
        "swept_over_naive": value / naive_value if naive_value else None,
        "effective_roofline_frac": value / (HBM_PEAK_GBS * 1e9 / NAIVE_BYTES[eq]),
        "roofline": roofline,
        "wall_ms_per_step": wall_ms,
        "with_host_copies": {"ms_per_step": paper_ms, "value": updates / (paper_ms * 1e-3),
                             "note": "one solve including device allocation and the host-to-device "
                                     "and device-to-host copies of the state (PCIe)"},
    }
    if not args.no_cpu_baseline:
        # one more solve from the same input, outside the timed region, for
        # the sampled check against the oracle in the CPU leg
        dev = solve_once(torch, eq, state0, work, width, threads, schedule)
        torch.cuda.synchronize()
        final = dev.cpu().numpy()
        del dev
        log("[bench] cpu baseline (oracle) and sampled check ...")
        out["cpu_baseline"] = cpu_baseline(work, eq, args.cpu_seconds, final)
        v = out["cpu_baseline"]["verify"]
        out["error_vs_oracle"] = {k: v[k] for k in v if k not in ("seconds",)}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
