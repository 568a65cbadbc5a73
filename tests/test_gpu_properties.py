"""Randomised GPU properties and the performance claim of the method.

* For random grid sizes that are a multiple of a random valid width, random
  workgroup sizes, random step counts (remainders included) and random
  initial states, the swept result equals the classic per-step result bit
  for bit, in every equation and precision.
* On the benchmark grids (2^22 cells) the swept rule is faster than the
  classic one-launch-per-step path, for heat and for Euler.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import paper_1811_08282_amd as sw
from paper_1811_08282_amd import workloads as wl
from gpu_util import announce, pack, run

pytestmark = pytest.mark.gpu

EQS = [sw.HEAT_F64, sw.HEAT_F32, sw.EULER_F64, sw.EULER_F32, sw.EULER_F64_FLAT,
       sw.EULER_F32_FLAT]


def _random_state(eq, n, seed):
    rng = np.random.default_rng(seed)
    if eq in (sw.HEAT_F64, sw.HEAT_F32):
        return pack(eq, rng.standard_normal(n))
    # smooth random gas state (a few periodic modes each): positive density
    # and pressure, moderate velocity, so no step leaves the physical range
    x = np.arange(n) / n

    def field(base, amp):
        k = rng.integers(1, 6, 3)
        a = rng.uniform(-1.0, 1.0, 3)
        ph = rng.uniform(0.0, 2 * np.pi, 3)
        f = sum(a[j] * np.sin(2 * np.pi * k[j] * x + ph[j]) for j in range(3)) / 3.0
        return base + amp * f

    rho = field(1.0, 0.5)
    vel = field(0.0, 0.3)
    p = field(1.0, 0.5)
    q = np.stack([rho, rho * vel, p / 0.4 + 0.5 * rho * vel * vel])
    layout = {sw.EULER_F64_FLAT: sw.EULER_F64, sw.EULER_F32_FLAT: sw.EULER_F32}.get(eq, eq)
    return pack(layout, q)


@st.composite
def _cases(draw):
    eq = draw(st.sampled_from(EQS))
    step = 2 * sw.radius(eq)
    if draw(st.booleans()):
        w = step * draw(st.integers(1, 128 // step))
        tiles = draw(st.integers(2, 9))
    else:  # the wide tiles of the default launches, compile-time widths included
        w = draw(st.sampled_from([256, 512, 1024, 2048]))
        tiles = draw(st.integers(2, 3))
    steps = draw(st.integers(0, min(3 * w, 700)))
    threads = draw(st.sampled_from([0, 64, 128, 256, 512]))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    return eq, w * tiles, w, steps, threads, seed


@settings(max_examples=150, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow])
@given(_cases())
def test_random_grids_swept_equals_naive(case):
    eq, n, w, steps, threads, seed = case
    announce("property", eq, n, w, steps, threads, seed)
    host = _random_state(eq, n, seed)
    dt = 0.25 if eq in (sw.HEAT_F64, sw.HEAT_F32) else 0.1
    swept = run(eq, host, steps, dt, 1.0, "swept", width=w, threads=threads)
    naive = run(eq, host, steps, dt, 1.0, "naive")
    assert np.array_equal(swept, naive), case


def _ms(eq, host, steps, dt, method):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    sw.solve(eq, t, steps, dt, 1.0, method=method)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    sw.solve(eq, t, steps, dt, 1.0, method=method)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b)


@pytest.mark.parametrize("name", ["heat", "euler"])
def test_swept_beats_naive_on_the_benchmark_grids(name):
    if name == "heat":
        w, eq, steps = wl.HEAT_LARGE, sw.HEAT_F64, 4000
        host = pack(eq, wl.initial_state(w))
    else:
        w, eq, steps = wl.EULER_LARGE, sw.EULER_F64, 500
        host = pack(eq, wl.initial_state(w))
    announce("swept vs naive timing", name, w.n, steps)
    swept = _ms(eq, host, steps, w.dt, "swept")
    naive = _ms(eq, host, steps, w.dt, "naive")
    print(f"[timing] {name}: swept {swept:.2f} ms, naive {naive:.2f} ms", flush=True)
    assert swept < naive
