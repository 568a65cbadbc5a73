"""Host logic of bench.py's sampled check against the oracle (no GPU).

A result computed by the oracle over the whole grid must pass the sampled
check bit for bit, and one wrong cell inside a sampled window, or in any
tile, must fail it.
"""
import numpy as np

import bench
import oracle
import paper_1811_08282_amd as sw
from paper_1811_08282_amd import workloads as wl

HEAT = wl.Workload("heat_n4096_s300", "heat", 4096, 300, 0.25, 1.0, 7)
EULER = wl.Workload("euler_n2048_s60", "euler", 2048, 60, 0.1, 1.0, None, 512)


def _full_heat_f64(work):
    u0 = wl.initial_state(work)
    return oracle.heat_f64(u0, work.steps, work.dt / work.dx ** 2).reshape(1, -1)


def test_heat_f64_sampled_check_passes_and_catches_a_wrong_cell():
    full = _full_heat_f64(HEAT)
    v = bench.verify_sample(HEAT, sw.HEAT_F64, full)
    assert v["bit_exact"] and v["max_abs_diff"] == 0.0
    bad = full.copy()
    bad[0, HEAT.n // 3 + 5 + 3] += 1e-12  # inside the second sampled window
    assert not bench.verify_sample(HEAT, sw.HEAT_F64, bad)["bit_exact"]


def test_heat_f32_sampled_check_states_its_binary64_error():
    u0 = wl.initial_state(HEAT).astype(np.float32)
    u, c = oracle.heat_f32(u0, np.zeros_like(u0), HEAT.steps, HEAT.dt / HEAT.dx ** 2)
    v = bench.verify_sample(HEAT, sw.HEAT_F32, np.stack([u, c]))
    assert v["bit_exact"]
    assert 0.0 < v["rel_inf_vs_binary64"] < 1e-6


def test_euler_sampled_check_covers_every_tile():
    q0 = wl.initial_state(EULER)
    full = oracle.euler_f64(q0, EULER.steps, EULER.dt / EULER.dx)
    v = bench.verify_sample(EULER, sw.EULER_F64, full)
    assert v["bit_exact"]
    bad = full.copy()
    bad[2, 3 * EULER.tile + 100] *= 1 + 1e-15
    assert not bench.verify_sample(EULER, sw.EULER_F64, bad)["bit_exact"]


def test_euler_f32_sampled_check_states_errors_per_variable():
    q0 = wl.initial_state(EULER).astype(np.float32)
    q, c = oracle.euler_f32(q0, np.zeros_like(q0), EULER.steps, EULER.dt / EULER.dx)
    v = bench.verify_sample(EULER, sw.EULER_F32, np.concatenate([q, c]))
    assert v["bit_exact"]
    assert set(v["rel_1_vs_binary64"]) == {"rho", "m", "E"}
    assert all(0.0 <= e < 1e-2 for e in v["rel_1_vs_binary64"].values())


def test_schedule_follows_the_library_route_rule():
    """bench.py times heat through one persistent launch exactly where
    swept_solve takes it: more than 1024 tiles of 1792 cells or more."""
    def work(eq, n):
        return wl.Workload(f"{eq}_{n}", eq, n, 10, 0.25, 1.0, 1)
    assert bench.default_schedule(sw.HEAT_F64, work("heat", 1 << 22)) == "persistent"
    assert bench.default_schedule(sw.HEAT_F32, work("heat", 1 << 24)) == "persistent"
    assert bench.default_schedule(sw.HEAT_F64, work("heat", 10_000_000)) == "persistent"  # W 2000
    assert bench.default_schedule(sw.HEAT_F64, work("heat", 1 << 21)) == "phases"  # 1024 tiles
    assert bench.default_schedule(sw.HEAT_F64, work("heat", 1 << 20)) == "phases"
    assert bench.default_schedule(sw.EULER_F64, work("euler", 1 << 24)) == "phases"
    assert bench.default_schedule(sw.KS_F64, work("ks", 1 << 24)) == "phases"
    assert not bench.persistent_route(sw.HEAT_F64, 1 << 23, 1024)  # narrow tiles
    assert bench.persistent_route(sw.HEAT_F64, 1792 * 1025, 1792)
    assert not bench.persistent_route(sw.HEAT_F64, 1792 * 1024, 1792)
