"""GPU parity at the benchmark configurations' full sizes.

At full size the oracle cannot step the whole grid in seconds, so each check
uses a property that holds at any size:

* heat: the value of cell j after n steps depends only on cells j-n..j+n, so
  the oracle stepping a window of 2n+3 (+ sample span) cells around a block of
  sampled cells computes those outputs exactly (the window's own periodic
  wrap cannot reach its centre within n steps);
* Euler on the Sod tiling: the initial state is periodic with the tile, so
  the solution is too, bit for bit -- the oracle steps one tile and every
  tile of the GPU result must equal it;
* swept == naive over the whole grid, bit for bit.

Every launch uses the triangle width bench.py times (the library default).
"""
import numpy as np
import pytest

import oracle
import paper_1811_08282_amd as sw
from paper_1811_08282_amd import workloads as wl
import batch_oracle as bo
from gpu_util import announce, pack, record, rel_inf, run

pytestmark = pytest.mark.gpu


def _heat_cone_samples(u0, steps, r, starts, span, fn):
    """Oracle values of cells [s, s+span) for each s in starts (periodic)."""
    n = u0.size
    out = {}
    for s in starts:
        idx = (np.arange(s - steps - 1, s + span + steps + 1)) % n
        res = fn(u0[idx], steps, r)
        out[s] = res[steps + 1: steps + 1 + span]
    return out


def _sample_starts(n):
    return [0, n // 3 + 5, n - 7, 12345 % n]


def test_heat_f64_n4194304_20000_steps():
    w = wl.HEAT_LARGE
    u0 = wl.initial_state(w)
    r = w.dt / w.dx ** 2
    announce("fullsize heat_f64 swept", w.n, w.steps)
    swept = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), w.steps, w.dt, w.dx, "swept")[0]
    announce("fullsize heat_f64 naive")
    naive = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), w.steps, w.dt, w.dx, "naive")[0]
    assert np.array_equal(swept, naive)
    span = 16
    ref = _heat_cone_samples(u0, w.steps, r, _sample_starts(w.n), span, oracle.heat_f64)
    for s, vals in ref.items():
        got = swept[(np.arange(s, s + span)) % w.n]
        assert np.array_equal(got, vals), s


def _persistent_solve(eq, host, work, threads=256):
    """One persistent launch of the heat-only batch holding the single
    problem, the launch bench.py times for heat grids (library width for a
    batch, 256-thread workgroups)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    torch.cuda.synchronize()
    b = sw.Batch([dict(eq=eq, width=0, n_cells=work.n, n_steps=work.steps, dt=work.dt,
                       dx=work.dx, d_state=t.data_ptr())], threads=threads)
    stream = torch.cuda.current_stream().cuda_stream
    b.run(stream)
    assert b.wait(stream) == sw.SW_OK, sw.last_error()
    width = b.width(0)
    b.close()
    return t.cpu().numpy(), width


@pytest.mark.parametrize("work,eq", [(wl.HEAT_LARGE, sw.HEAT_F64), (wl.HEAT_PREC, sw.HEAT_F64),
                                     (wl.HEAT_PREC, sw.HEAT_F32)],
                         ids=["f64_n4194304", "f64_n16777216", "f32_n16777216"])
def test_persistent_heat_launch_whole_grid(work, eq):
    """The benchmarked heat launch at its benchmark size: one persistent
    launch of W = 2048 tiles (2048 or 8192 tiles per phase, 21 overlapping
    phases, every XCD taking tiles of every phase) equals naive_solve over
    the whole grid bit for bit, and the oracle on dependency-cone windows."""
    u0 = wl.initial_state(work)
    host = pack(eq, u0)
    announce("fullsize persistent heat", eq, work.n, work.steps)
    got, width = _persistent_solve(eq, host, work)
    assert width == 2048
    announce("fullsize persistent heat: naive", eq, work.n, work.steps)
    naive = run(eq, host, work.steps, work.dt, work.dx, "naive")
    assert np.array_equal(got, naive)
    r = work.dt / work.dx ** 2
    span = 16
    starts = _sample_starts(work.n)
    if eq == sw.HEAT_F64:
        ref = _heat_cone_samples(u0, work.steps, r, starts, span, oracle.heat_f64)
        for s0, vals in ref.items():
            assert np.array_equal(got[0][(np.arange(s0, s0 + span)) % work.n], vals), s0
    else:
        u32 = u0.astype(np.float32)
        zero_c = np.zeros(work.n, np.float32)
        for s0 in starts:
            idx = (np.arange(s0 - work.steps - 1, s0 + span + work.steps + 1)) % work.n
            u, c = oracle.heat_f32(u32[idx], zero_c[idx], work.steps, r)
            sel = (np.arange(s0, s0 + span)) % work.n
            assert np.array_equal(got[0][sel], u[work.steps + 1: work.steps + 1 + span]), s0
            assert np.array_equal(got[1][sel], c[work.steps + 1: work.steps + 1 + span]), s0


def test_euler_f64_n4194304_10000_steps():
    w = wl.EULER_LARGE
    q0 = wl.initial_state(w)
    announce("fullsize euler_f64 swept", w.n, w.steps)
    swept = run(sw.EULER_F64, pack(sw.EULER_F64, q0), w.steps, w.dt, w.dx, "swept")
    announce("fullsize euler_f64 naive")
    naive = run(sw.EULER_F64, pack(sw.EULER_F64, q0), w.steps, w.dt, w.dx, "naive")
    assert np.array_equal(swept, naive)
    tile = oracle.euler_f64(q0[:, :w.tile], w.steps, w.dt / w.dx)
    tiles = swept.reshape(3, w.n // w.tile, w.tile)
    record("euler_f64_n4194304_s10000_vs_oracle",
           max_abs_diff=float(np.max(np.abs(tiles - tile[:, None, :]))))
    assert np.array_equal(tiles, np.broadcast_to(tile[:, None, :], tiles.shape))


def test_euler_f64_flat_n4194304_10000_steps():
    """The flattened layout at full size equals the oracle tile bit for bit."""
    w = wl.EULER_LARGE
    q0 = wl.initial_state(w)
    announce("fullsize euler_f64_flat swept", w.n, w.steps)
    swept = run(sw.EULER_F64_FLAT, pack(sw.EULER_F64, q0), w.steps, w.dt, w.dx, "swept")
    announce("fullsize euler_f64_flat naive")
    naive = run(sw.EULER_F64_FLAT, pack(sw.EULER_F64, q0), w.steps, w.dt, w.dx, "naive")
    assert np.array_equal(swept, naive)
    tile = oracle.euler_f64(q0[:, :w.tile], w.steps, w.dt / w.dx)
    tiles = swept.reshape(3, w.n // w.tile, w.tile)
    assert np.array_equal(tiles, np.broadcast_to(tile[:, None, :], tiles.shape))


def test_heat_f32_n16777216_20000_steps_error_vs_f64():
    w = wl.HEAT_PREC
    u0 = wl.initial_state(w)
    r = w.dt / w.dx ** 2
    announce("fullsize heat_f32 swept", w.n, w.steps)
    swept = run(sw.HEAT_F32, pack(sw.HEAT_F32, u0), w.steps, w.dt, w.dx, "swept")
    announce("fullsize heat_f32 naive")
    naive = run(sw.HEAT_F32, pack(sw.HEAT_F32, u0), w.steps, w.dt, w.dx, "naive")
    assert np.array_equal(swept, naive)
    u32 = u0.astype(np.float32)
    span = 16
    starts = _sample_starts(w.n)
    zero_c = np.zeros(w.n, np.float32)
    for s in starts:
        idx = (np.arange(s - w.steps - 1, s + span + w.steps + 1)) % w.n
        u, c = oracle.heat_f32(u32[idx], zero_c[idx], w.steps, r)
        sel = (np.arange(s, s + span)) % w.n
        assert np.array_equal(swept[0][sel], u[w.steps + 1: w.steps + 1 + span])
        assert np.array_equal(swept[1][sel], c[w.steps + 1: w.steps + 1 + span])
    # stated error of binary32 + Kahan against binary64 from the same rounded IC
    ref = _heat_cone_samples(u32.astype(np.float64), w.steps, r, starts, span, oracle.heat_f64)
    got = np.concatenate([swept[0][(np.arange(s, s + span)) % w.n] for s in starts])
    want = np.concatenate([ref[s] for s in starts])
    err = rel_inf(got, want)
    record("heat_f32_n16777216_s20000_vs_f64", rel_inf=err, cells=int(got.size))
    assert err < 1e-6


def test_euler_f32_n16777216_20000_steps_error_vs_f64():
    w = wl.EULER_PREC
    q0 = wl.initial_state(w)
    announce("fullsize euler_f32 swept", w.n, w.steps)
    swept = run(sw.EULER_F32, pack(sw.EULER_F32, q0), w.steps, w.dt, w.dx, "swept")
    announce("fullsize euler_f32 naive")
    naive = run(sw.EULER_F32, pack(sw.EULER_F32, q0), w.steps, w.dt, w.dx, "naive")
    assert np.array_equal(swept, naive)
    q32 = q0[:, :w.tile].astype(np.float32)
    tq, tc = oracle.euler_f32(q32, np.zeros_like(q32), w.steps, w.dt / w.dx)
    tiles = swept.reshape(6, w.n // w.tile, w.tile)
    want = np.concatenate([tq, tc])
    assert np.array_equal(tiles, np.broadcast_to(want[:, None, :], tiles.shape))
    # stated error against binary64 from the binary32-rounded IC (limiter switching
    # dominates: rel_1 of rho and E, the smooth-norm measures, are gated)
    ref = oracle.euler_f64(q32.astype(np.float64), w.steps, w.dt / w.dx)
    rel1 = np.abs(tq - ref).sum(axis=1) / np.abs(ref).sum(axis=1)
    record("euler_f32_n16777216_s20000_vs_f64", rel_1=rel1.tolist(),
           rel_inf=[rel_inf(tq[k], ref[k]) for k in range(3)])
    assert rel1[0] < 1e-2 and rel1[2] < 1e-2


def test_heat_f64_beyond_2_31_cells():
    """A grid of 2^31 + 2^29 cells (cell offsets past the 32-bit range; 21 GB
    of state, 86 GB of swept working arrays): swept and classic against the
    oracle on dependency cones at the start, across 2^31 and at the periodic
    seam.  The initial state is dyadic and generated on the device by integer
    arithmetic that the host repeats exactly for the sampled windows."""
    import torch
    n, steps, r = (1 << 31) + (1 << 29), 600, 0.25

    def ic_host(idx):
        return ((idx.astype(np.int64) * 40503) % 1021).astype(np.float64) / 1024.0

    def ic_device():
        j = torch.arange(n, dtype=torch.int64, device="cuda")
        j.mul_(40503).remainder_(1021)
        u = j.to(torch.float64).div_(1024.0)
        del j
        return u.reshape(1, n)

    span = 16
    starts = [0, (1 << 31) - 8, n - 8]
    want = {}
    for s0 in starts:
        idx = np.arange(s0 - steps - 1, s0 + span + steps + 1) % n
        want[s0] = oracle.heat_f64(ic_host(idx), steps, r)[steps + 1: steps + 1 + span]
    for method in ("swept", "naive"):
        announce("beyond 2^31 cells heat_f64", method, n, steps)
        u = ic_device()
        sw.solve(sw.HEAT_F64, u, steps, r, 1.0, method=method)
        torch.cuda.synchronize()
        for s0 in starts:
            sel = torch.arange(s0, s0 + span, device="cuda") % n
            got = u[0, sel].cpu().numpy()
            assert np.array_equal(got, want[s0]), (method, s0)
        del u
        sw.sw_release()
        torch.cuda.empty_cache()


def test_euler_f32_flat_n16777216_20000_steps():
    """The flattened binary32 layout at full size (the launch bench.py times:
    W = 2048, 512-thread workgroups) equals the binary32 oracle tile bit for
    bit, and so the lengthened binary32 result."""
    w = wl.EULER_PREC
    q0 = wl.initial_state(w)
    assert sw.sw_default_width(sw.EULER_F32_FLAT, w.n) == 2048
    announce("fullsize euler_f32_flat swept", w.n, w.steps)
    swept = run(sw.EULER_F32_FLAT, pack(sw.EULER_F32, q0), w.steps, w.dt, w.dx, "swept")
    q32 = q0[:, :w.tile].astype(np.float32)
    tq, tc = oracle.euler_f32(q32, np.zeros_like(q32), w.steps, w.dt / w.dx)
    tiles = swept.reshape(6, w.n // w.tile, w.tile)
    want = np.concatenate([tq, tc])
    assert np.array_equal(tiles, np.broadcast_to(want[:, None, :], tiles.shape))


_BATCH_CHOICE = {}  # precision -> (widths, blocks_per_cu, threads) chosen by the tuning test


def _batch_specs(eq_heat, eq_euler):
    import torch
    probs = wl.batch_problems()
    tensors, hosts, specs = [], [], []
    for p in probs:
        eq = eq_heat if p.eq == "heat" else eq_euler
        host = pack(eq, wl.batch_ic(p))
        t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
        dt, dx = (0.25, 1.0) if p.eq == "heat" else (0.1, 1.0)
        tensors.append(t)
        hosts.append(host)
        specs.append(dict(eq=eq, width=0, n_cells=p.n, n_steps=5000, dt=dt, dx=dx,
                          d_state=t.data_ptr()))
    torch.cuda.synchronize()
    return probs, tensors, hosts, specs


def _time_run(b, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    b.run(stream)
    stop.record()
    assert b.wait(stream) == sw.SW_OK, sw.last_error()
    return start.elapsed_time(stop)


@pytest.mark.parametrize("eq_heat,eq_euler", [(sw.HEAT_F64, sw.EULER_F64),
                                              (sw.HEAT_F32, sw.EULER_F32)])
def test_batch_4096_problems_autotune(eq_heat, eq_euler):
    """The batch autotuner on the full batched workload (4096 problems,
    lengths log-uniform in [2^10, 2^18], half heat / half Euler, 5000 steps),
    once per workgroup size with short probes; the two tuned launches are
    then timed at full length and the faster is kept for the next test.  The
    caller's states are only read."""
    import torch
    probs, tensors, hosts, specs = _batch_specs(eq_heat, eq_euler)
    stream = torch.cuda.current_stream().cuda_stream
    timed = []
    for size in (256, 512):
        cand = [dict(s) for s in specs]
        announce("fullsize batch autotune", eq_heat, "threads", size)
        bpc, threads, per_update = sw.sw_batch_autotune(cand, 100, threads=size)
        b = sw.Batch(cand, blocks_per_cu=bpc, threads=threads)
        ms = _time_run(b, stream)   # advances the states; the next test starts afresh
        b.close()
        announce("tuned", threads, "blocks/CU", bpc, "full run ms", ms)
        timed.append((ms, [c["width"] for c in cand], bpc, threads))
    ms, widths, bpc, threads = min(timed)
    _BATCH_CHOICE[sw.is_f64(eq_heat)] = (widths, bpc, threads)
    record(f"batch_4096x5000_{'f64' if sw.is_f64(eq_heat) else 'f32'}_tuning",
           full_run_ms={str(t[3]): t[0] for t in timed}, chosen_threads=threads)


@pytest.mark.parametrize("eq_heat,eq_euler", [(sw.HEAT_F64, sw.EULER_F64),
                                              (sw.HEAT_F32, sw.EULER_F32)])
def test_batch_4096_problems_5000_steps(eq_heat, eq_euler):
    """The batched workload at full size in one persistent launch, with the
    launch the tuning test chose (the library defaults if it did not run).
    Every problem must equal its own swept solve (phase launches, a different
    schedule of the same tile bodies).  128 problems drawn across the length
    range, the longest heat and Euler problems among them, must equal the
    oracle (whole problems, or exact dependency-cone windows of the long
    ones): through the digests tests/golden/make_batch_oracle.py stored from
    the oracle, and the two longest also against the oracle stepped live on
    the host threads while the GPU works.
    (A classic solve of every problem would take 2 * 10^7 launches.)"""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    pair = "f64" if sw.is_f64(eq_heat) else "f32"
    probs, tensors, hosts, specs = _batch_specs(eq_heat, eq_euler)
    golden = bo.load_golden()
    assert golden["steps"] == 5000
    rows = golden["pairs"][pair]["problems"]
    subset = bo.subset(probs)
    assert len(subset) >= 120
    assert subset == golden["pairs"][pair]["subset"], \
        "the batch subset changed: rerun tests/golden/make_batch_oracle.py"
    for r in rows:
        assert probs[r["problem"]].n == r["n"] and specs[r["problem"]]["eq"] == r["eq"], \
            "the batched workload changed: rerun tests/golden/make_batch_oracle.py"
    live = [max((i for i in subset if probs[i].eq == kind), key=lambda i: probs[i].n)
            for kind in ("heat", "euler")]
    pool = ThreadPoolExecutor(max_workers=1)
    futures = {i: pool.submit(bo.sample, specs[i]["eq"], hosts[i], 5000, 15) for i in live}
    widths, bpc, threads = _BATCH_CHOICE.get(sw.is_f64(eq_heat), (None, 0, 0))
    if widths:
        for s, w in zip(specs, widths):
            s["width"] = w
    announce("fullsize batch", eq_heat, eq_euler, "problems", len(specs), "blocks/CU", bpc,
             "threads", threads, "oracle subset", len(subset))
    b = sw.Batch(specs, blocks_per_cu=bpc, threads=threads)
    stream = torch.cuda.current_stream().cuda_stream
    b.run(stream)
    assert b.wait(stream) == sw.SW_OK, sw.last_error()
    widths = [b.width(i) for i in range(len(specs))]
    finals = {i: tensors[i].cpu().numpy() for i in subset}
    # every problem solved alone (phase launches) from the same initial state,
    # all enqueued at once, compared with the batch result on the device
    announce("fullsize batch: every problem alone")
    alone = [torch.from_numpy(np.ascontiguousarray(h)).cuda() for h in hosts]
    for i, s in enumerate(specs):
        sw.solve(s["eq"], alone[i], 5000, s["dt"], s["dx"], method="swept", width=widths[i])
    torch.cuda.synchronize()
    differ = [i for i in range(len(specs)) if not torch.equal(tensors[i], alone[i])]
    assert not differ, differ[:10]
    del alone
    # throughput of one more replay of the captured launch (5000 further steps)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    b.run(stream)
    stop.record()
    assert b.wait(stream) == sw.SW_OK, sw.last_error()
    ms = start.elapsed_time(stop)
    cells = sum(p.n for p in probs)
    b.close()
    # the oracle digests of all 128
    checked_widths = set()
    bad = []
    for r in rows:
        i = r["problem"]
        vals = finals[i][:, bo.sample_cells(specs[i]["eq"], probs[i].n)]
        assert vals.shape[1] == r["cells"]
        if bo.digest(vals) != r["sha256"]:
            bad.append((i, probs[i].n, widths[i], [float(x).hex() for x in vals[:, 0]], r["first"]))
        checked_widths.add((probs[i].eq, widths[i]))
    assert not bad, bad[:4]
    announce("fullsize batch: oracle digests of", len(rows), "problems equal; live oracle")
    for i in live:
        sampled, want = futures[i].result()
        assert np.array_equal(finals[i][:, sampled], want), (i, probs[i].n, widths[i])
    pool.shutdown()
    tag = 'f64' if sw.is_f64(eq_heat) else 'f32'
    record(f"batch_4096x5000_{tag}", ms=ms, cells=cells,
           cell_updates_per_s=cells * 5000 / (ms * 1e-3), blocks_per_cu=bpc, threads=threads,
           distinct_widths=len(set(widths)), widest=max(widths), narrowest=min(widths),
           oracle_checked=len(rows), oracle_live=len(live), oracle_widths=sorted(checked_widths))
    # the widest tile of each equation in the batch was among the oracle checks
    for kind in ("heat", "euler"):
        wmax = max(w for p, w in zip(probs, widths) if (p.eq == "heat") == (kind == "heat"))
        assert any(w == wmax and (e == "heat") == (kind == "heat") for e, w in checked_widths)
