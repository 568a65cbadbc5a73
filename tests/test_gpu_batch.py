"""GPU tests of the batched persistent launch and of the autotuner.

A problem solved inside a batch must be bit-identical to the same problem
solved alone by swept_solve with the same width (the same tile-phase code
runs in both), and hence to the oracle.
"""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import oracle
import paper_1811_08282_amd as sw
from paper_1811_08282_amd.workloads import heat_ic, sod_tiled
from gpu_util import announce, pack, run

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ic(eq, n, seed):
    if eq in (sw.HEAT_F64, sw.HEAT_F32):
        return heat_ic(n, seed)
    return sod_tiled(n, n)


def _pack_eq(eq):
    """state layout of the flattened ids equals the lengthened ones"""
    return {sw.EULER_F64_FLAT: sw.EULER_F64, sw.EULER_F32_FLAT: sw.EULER_F32}.get(eq, eq)


def _coef(eq):
    return (0.25, 1.0) if eq in (sw.HEAT_F64, sw.HEAT_F32) else (0.1, 1.0)


def _problems(specs):
    """specs: (eq, n, steps, width, seed) -> (device tensors, host ICs, sw_problem dicts)"""
    import torch
    tensors, hosts, probs = [], [], []
    for eq, n, steps, width, seed in specs:
        host = pack(_pack_eq(eq), _ic(eq, n, seed))
        t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
        dt, dx = _coef(eq)
        tensors.append(t)
        hosts.append(host)
        probs.append(dict(eq=eq, width=width, n_cells=n, n_steps=steps, dt=dt, dx=dx,
                          d_state=t.data_ptr()))
    torch.cuda.synchronize()
    return tensors, hosts, probs


MIXED = [
    (sw.HEAT_F64, 1024, 300, 64, 1),
    (sw.HEAT_F32, 2048, 1, 128, 2),      # single phase: copy-out items
    (sw.EULER_F64, 2048, 50, 256, 3),
    (sw.EULER_F32, 1024, 30, 64, 4),
    (sw.HEAT_F64, 4096, 0, 64, 5),       # no work
    (sw.HEAT_F64, 1000, 77, 40, 6),      # ragged width
    (sw.EULER_F64, 512, 9, 2, 7),        # width 2: one level per phase
    (sw.HEAT_F32, 8192, 333, 1024, 8),
    (sw.EULER_F64_FLAT, 2048, 41, 128, 9),   # flattened layout, radius-2 halos
    (sw.EULER_F32_FLAT, 1024, 17, 4, 10),
    (sw.EULER_F64, 3072, 300, 1024, 11),     # compile-time widths of both workgroup sizes
    (sw.EULER_F32, 2048, 200, 512, 12),
]


@pytest.mark.parametrize("threads", [0, 512])
def test_mixed_batch_equals_individual_swept_and_oracle(threads):
    import torch
    tensors, hosts, probs = _problems(MIXED)
    announce("batch mixed", len(probs), "threads", threads)
    b = sw.Batch(probs, threads=threads)
    items, blocks, nbytes = b.info()
    assert items > 0 and blocks > 0
    b.run(torch.cuda.current_stream().cuda_stream)
    assert b.wait(torch.cuda.current_stream().cuda_stream) == sw.SW_OK, sw.last_error()
    for (eq, n, steps, width, seed), t, host in zip(MIXED, tensors, hosts):
        got = t.cpu().numpy()
        dt, dx = _coef(eq)
        announce("batch check", eq, n, steps, width)
        alone = run(eq, host, steps, dt, dx, "swept", width=width)
        assert np.array_equal(got, alone), (eq, n, steps, width)
        if eq == sw.HEAT_F64:
            assert np.array_equal(got[0], oracle.heat_f64(host[0], steps, dt / dx ** 2))
        elif eq in (sw.EULER_F64, sw.EULER_F64_FLAT):
            assert np.array_equal(got, oracle.euler_f64(host, steps, dt / dx))
        elif eq == sw.HEAT_F32:
            u, c = oracle.heat_f32(host[0], host[1], steps, dt / dx ** 2)
            assert np.array_equal(got[0], u) and np.array_equal(got[1], c)
        else:
            q, c = oracle.euler_f32(host[:3], host[3:], steps, dt / dx)
            assert np.array_equal(got[:3], q) and np.array_equal(got[3:], c)
    b.close()


def test_graph_replays_match_eager_runs():
    """Replay the captured graph three times with eager solves and host
    synchronisation between the replays; every replay must match."""
    import torch
    specs = [(sw.HEAT_F64, 2048, 97, 128, 11), (sw.EULER_F64, 1024, 13, 64, 12),
             (sw.HEAT_F32, 1024, 40, 64, 13)]
    tensors, hosts, probs = _problems(specs)
    b = sw.Batch(probs)
    eager = [h.copy() for h in hosts]
    stream = torch.cuda.current_stream().cuda_stream
    for rep in range(3):
        announce("batch replay", rep)
        b.run(stream)
        assert b.wait(stream) == sw.SW_OK, sw.last_error()
        for i, (eq, n, steps, width, seed) in enumerate(specs):
            dt, dx = _coef(eq)
            eager[i] = run(eq, eager[i], steps, dt, dx, "swept", width=width)
            assert np.array_equal(tensors[i].cpu().numpy(), eager[i]), (rep, i)
    b.close()


def _batch_ws(probs):
    import torch
    nbytes = sw.sw_batch_workspace_bytes(probs)
    assert nbytes > 0, sw.last_error()
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    assert ws.data_ptr() % 256 == 0
    return ws, nbytes


def test_default_widths_and_one_shot_entry_point():
    """swept_solve_batch in a caller workspace, library-chosen widths: every
    problem equals its own swept solve; a second call with a smaller list
    reuses the same workspace."""
    import torch
    specs = [(sw.HEAT_F64, 256 * 5, 50, 0, 21), (sw.EULER_F32, 256 * 6, 20, 0, 22),
             (sw.EULER_F64_FLAT, 256 * 4, 33, 0, 23)]
    tensors, hosts, probs = _problems(specs)
    ws, nbytes = _batch_ws(probs)
    stream = torch.cuda.current_stream().cuda_stream
    announce("batch one-shot", len(probs))
    assert sw.swept_solve_batch(probs, ws.data_ptr(), nbytes, stream) == sw.SW_OK, sw.last_error()
    assert sw.sw_batch_check(ws.data_ptr(), stream) == sw.SW_OK
    for (eq, n, steps, width, seed), t, host in zip(specs, tensors, hosts):
        dt, dx = _coef(eq)
        alone = run(eq, host, steps, dt, dx, "swept")
        assert np.array_equal(t.cpu().numpy(), alone)
    small = [(sw.HEAT_F32, 512, 70, 0, 24)]
    tensors, hosts, probs = _problems(small)
    announce("batch one-shot, smaller list in the same workspace")
    assert sw.swept_solve_batch(probs, ws.data_ptr(), nbytes, stream) == sw.SW_OK, sw.last_error()
    assert sw.sw_batch_check(ws.data_ptr(), stream) == sw.SW_OK
    alone = run(sw.HEAT_F32, hosts[0], 70, 0.25, 1.0, "swept")
    assert np.array_equal(tensors[0].cpu().numpy(), alone)


@pytest.mark.parametrize("threads", [0, 512])
def test_swept_solve_batch_captured_in_a_graph(threads):
    """swept_solve_batch captured into a HIP graph (table upload, reset and
    persistent kernels): the capture runs nothing, and each of three replays,
    with eager solves and host synchronisation between them, equals the same
    number of eager solves of every problem."""
    import torch
    specs = [(sw.HEAT_F64, 2048, 97, 128, 81), (sw.EULER_F64, 1024, 13, 64, 82),
             (sw.HEAT_F32, 1024, 1, 64, 83), (sw.EULER_F32_FLAT, 2048, 9, 256, 84)]
    tensors, hosts, probs = _problems(specs)
    ws, nbytes = _batch_ws(probs)
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    announce("batch graph capture", threads)
    with torch.cuda.graph(graph, stream=stream):
        rc = sw.swept_solve_batch(probs, ws.data_ptr(), nbytes,
                                  torch.cuda.current_stream().cuda_stream, threads=threads)
    assert rc == sw.SW_OK, sw.last_error()
    torch.cuda.synchronize()
    for t, h in zip(tensors, hosts):
        assert np.array_equal(t.cpu().numpy(), h)  # capture runs nothing
    eager = [h.copy() for h in hosts]
    for rep in range(3):
        announce("batch graph replay", rep)
        graph.replay()
        torch.cuda.synchronize()
        assert sw.sw_batch_check(ws.data_ptr(), None) == sw.SW_OK
        for i, (eq, n, steps, width, seed) in enumerate(specs):
            dt, dx = _coef(eq)
            eager[i] = run(eq, eager[i], steps, dt, dx, "swept", width=width)
            assert np.array_equal(tensors[i].cpu().numpy(), eager[i]), (rep, i)


def test_bounded_wait_aborts_cleanly():
    """A 1-microsecond bound on dependency waits makes the launch give up;
    every workgroup leaves and the failure is reported, then a normal batch
    still runs."""
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    tensors, hosts, probs = _problems([(sw.HEAT_F64, 128, 3000, 64, 31)])
    announce("batch forced abort")
    b = sw.Batch(probs, wait_limit_us=1)
    b.run(stream)
    rc = b.wait(stream)
    assert rc == sw.SW_ERR_HIP and "time bound" in sw.last_error()
    b.close()
    tensors, hosts, probs = _problems([(sw.HEAT_F64, 128, 300, 64, 32)])
    b = sw.Batch(probs)
    b.run(stream)
    assert b.wait(stream) == sw.SW_OK
    alone = run(sw.HEAT_F64, hosts[0], 300, 0.25, 1.0, "swept", width=64)
    assert np.array_equal(tensors[0].cpu().numpy(), alone)
    b.close()


def test_batch_rejects_bad_problems():
    import torch
    t = torch.zeros(1, 1024, dtype=torch.float64, device="cuda")
    bad = [dict(eq=sw.HEAT_F64, width=48, n_cells=1024, n_steps=5, dt=0.25, dx=1.0,
                d_state=t.data_ptr())]
    with pytest.raises(sw.SweptError):
        sw.Batch(bad)
    bad[0]["width"] = 64
    with pytest.raises(sw.SweptError):
        sw.Batch(bad, threads=128)  # the batch kernel has 256- and 512-thread forms only
    bad[0]["dt"] = -1.0
    with pytest.raises(sw.SweptError):
        sw.Batch(bad)


# ---- autotuner -------------------------------------------------------------------

def test_autotune_records_and_is_used():
    sw.sw_tune_clear()
    n = 1 << 16
    announce("autotune heat_f64", n)
    w, threads, ms = sw.sw_autotune(sw.HEAT_F64, n, 0)
    assert w % 64 == 0 and n % w == 0 and n // w >= 2 and threads in (64, 128, 256, 512)
    assert ms > 0
    assert sw.sw_tuned_width(sw.HEAT_F64, n) == (w, threads)
    # a cell count of the same size class with no record of its own takes it
    import torch
    n2 = n + n // 4
    t2 = torch.zeros(1, n2, dtype=torch.float64, device="cuda")
    b = sw.Batch([dict(eq=sw.HEAT_F64, width=0, n_cells=n2, n_steps=1, dt=0.25, dx=1.0,
                       d_state=t2.data_ptr())])
    if n2 % w == 0 and n2 // w >= 2:
        assert b.width(0) == w
    else:  # the batch's own default: the largest valid heat width up to 2048
        assert b.width(0) == max(v for v in range(2, 2049, 2) if n2 % v == 0 and n2 // v >= 2)
    b.close()
    u0 = heat_ic(n, 41)
    got = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), 333, 0.25, 1.0, "swept")[0]
    assert np.array_equal(got, oracle.heat_f64(u0, 333, 0.25))
    announce("autotune euler_f32")
    w2, t2, _ = sw.sw_autotune(sw.EULER_F32, 4096, 8)
    assert 4096 % w2 == 0
    sw.sw_tune_clear()
    assert sw.sw_tuned_width(sw.HEAT_F64, n) is None


def test_autotune_cache_file_persists_across_processes():
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        env = dict(os.environ, SWEPT_TUNE_CACHE=path, PYTHONPATH=ROOT)
        code_a = ("import paper_1811_08282_amd as sw; "
                  "print(sw.sw_autotune(sw.HEAT_F64, 8192, 64)[:2])")
        code_b = ("import paper_1811_08282_amd as sw; print(sw.sw_tuned_width(sw.HEAT_F64, 8192))")
        announce("autotune cache file")
        a = subprocess.run([sys.executable, "-c", code_a], env=env, capture_output=True, text=True,
                           timeout=120)
        assert a.returncode == 0, a.stderr
        b = subprocess.run([sys.executable, "-c", code_b], env=env, capture_output=True, text=True,
                           timeout=120)
        assert b.returncode == 0, b.stderr
        assert a.stdout.strip() == b.stdout.strip()
        assert open(path).read().split()[0].startswith("gfx")


def test_batch_autotune_picks_widths_and_workgroups_reading_states_only():
    """sw_batch_autotune writes a valid width into every problem given with
    width 0, picks a resident-workgroup count, leaves the caller's states as
    they were, and a batch built with its choices still matches the
    individual solves."""
    import torch
    specs = [(sw.HEAT_F64, 256 * 5, 40, 0, 51), (sw.HEAT_F64, 256 * 6, 40, 0, 52),
             (sw.EULER_F32, 256 * 8, 12, 0, 53), (sw.EULER_F32, 256 * 12, 12, 64, 54),
             (sw.EULER_F64_FLAT, 256 * 8, 9, 0, 55)]
    tensors, hosts, probs = _problems(specs)
    announce("batch autotune")
    bpc, threads, ms = sw.sw_batch_autotune(probs, 8)
    assert bpc >= 0 and threads in (256, 512) and ms > 0
    for t, h in zip(tensors, hosts):
        assert np.array_equal(t.cpu().numpy(), h)  # read only
    assert probs[3]["width"] == 64  # a width given by the caller is kept
    for p in probs:
        w = p["width"]
        step = 2 * sw.radius(p["eq"])
        assert w > 0 and w % step == 0 and p["n_cells"] % w == 0 and p["n_cells"] // w >= 2
    b = sw.Batch(probs, blocks_per_cu=bpc, threads=threads)
    stream = torch.cuda.current_stream().cuda_stream
    b.run(stream)
    assert b.wait(stream) == sw.SW_OK, sw.last_error()
    for i, ((eq, n, steps, width, seed), t, host) in enumerate(zip(specs, tensors, hosts)):
        assert b.width(i) == probs[i]["width"]
        dt, dx = _coef(eq)
        alone = run(eq, host, steps, dt, dx, "swept", width=b.width(i))
        assert np.array_equal(t.cpu().numpy(), alone), i
    b.close()


@pytest.mark.parametrize("eq", [sw.HEAT_F64, sw.EULER_F64, sw.EULER_F32_FLAT])
def test_swept_solve_captured_in_a_graph(eq):
    """swept_solve_ex with a caller workspace captured into a HIP graph: three
    replays, with eager solves and host synchronisation between them, each
    equal to the same number of eager solves."""
    import torch
    n, steps = 4096, 150
    if eq == sw.HEAT_F64:
        host, dt = pack(eq, heat_ic(n, 71)), 0.25
    else:
        host, dt = pack(_pack_eq(eq), sod_tiled(n, 1024)), 0.1
    nbytes = sw.sw_workspace_bytes(eq, n)
    ws = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device="cuda")
    assert ws.data_ptr() % 256 == 0
    state = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    announce("graph capture", eq)
    with torch.cuda.graph(graph, stream=stream):
        sw.solve(eq, state, steps, dt, 1.0, workspace=ws)
    torch.cuda.synchronize()
    assert np.array_equal(state.cpu().numpy(), host)  # capture runs nothing
    eager = host.copy()
    for rep in range(3):
        announce("graph replay", eq, rep)
        graph.replay()
        torch.cuda.synchronize()
        eager = run(eq, eager, steps, dt, 1.0, "swept")
        assert np.array_equal(state.cpu().numpy(), eager), rep


@pytest.mark.parametrize("eq", [sw.HEAT_F64, sw.HEAT_F32])
@pytest.mark.parametrize("threads", [0, 512])
def test_heat_only_batch_runs_the_heat_kernel_and_matches(eq, threads):
    """A batch whose problems are all heat of one precision runs the
    persistent kernel compiled with that body alone; every problem (one-step
    copy-out items, ragged widths and remainders included) still equals its
    own swept solve and the oracle bit for bit."""
    import torch
    specs = [(eq, 2048, 1, 256, 61),      # single phase: copy-out items
             (eq, 1000, 77, 40, 62),      # ragged width
             (eq, 3 * 2048, 1500, 2048, 63),
             (eq, 4096, 333, 1024, 64),
             (eq, 4098, 100, 2, 65)]      # one level per phase
    tensors, hosts, probs = _problems(specs)
    announce("heat-only batch", eq, "threads", threads)
    b = sw.Batch(probs, threads=threads)
    stream = torch.cuda.current_stream().cuda_stream
    b.run(stream)
    assert b.wait(stream) == sw.SW_OK, sw.last_error()
    for (e, n, steps, width, seed), t, host in zip(specs, tensors, hosts):
        got = t.cpu().numpy()
        alone = run(e, host, steps, 0.25, 1.0, "swept", width=width)
        assert np.array_equal(got, alone), (n, steps, width)
        if e == sw.HEAT_F64:
            assert np.array_equal(got[0], oracle.heat_f64(host[0], steps, 0.25))
        else:
            u, c = oracle.heat_f32(host[0], host[1], steps, 0.25)
            assert np.array_equal(got[0], u) and np.array_equal(got[1], c)
    b.close()
