"""Kuramoto-Sivashinsky on the GPU through the C ABI against the oracle, bit
for bit: the classic kernel, the swept schedule at every width (radius-2
geometry: multiples of 4), ragged grids and every workgroup size, chunked
calls and cyclic shifts, and the full 2^24-cell x 20000-step workload (swept
== classic over the whole grid, the oracle on exact dependency cones of
radius 2 per step)."""
import numpy as np
import pytest

import oracle
import paper_1811_08282_amd as sw
from paper_1811_08282_amd import workloads as wl
from paper_1811_08282_amd.workloads import ks_ic
from gpu_util import announce, run

pytestmark = pytest.mark.gpu
DT, DX = 0.02, 1.0


def _u0(n, seed):
    return ks_ic(n, seed)


@pytest.mark.parametrize("n", [1000, 1024])
def test_ks_naive_equals_oracle(n):
    u0 = _u0(n, n)
    announce("ks naive", n)
    got = run(sw.KS_F64, u0.reshape(1, -1), 300, DT, DX, "naive")[0]
    assert np.array_equal(got, oracle.ks_f64(u0, 300, DT, DX))


@pytest.mark.parametrize("width", [4, 8, 16, 64, 128, 256, 512, 1024])
def test_ks_swept_every_width(width):
    n = 2048
    u0 = _u0(n, 3)
    rng = np.random.default_rng(width)
    h = width // 4
    for steps in sorted({1, h, h + 1, 3 * width + 5, int(rng.integers(1, 600))}):
        announce("ks swept W", width, "steps", steps)
        got = run(sw.KS_F64, u0.reshape(1, -1), steps, DT, DX, "swept", width=width)[0]
        assert np.array_equal(got, oracle.ks_f64(u0, steps, DT, DX)), (width, steps)


@pytest.mark.parametrize("n,width,threads", [(1000, 40, 0), (1000, 200, 64), (1200, 12, 0),
                                             (4 * 2048, 0, 0),
                                             (2 * 8192, 8192, 256), (6144, 1024, 512),
                                             (6144, 2048, 128)])
def test_ks_ragged_shapes_and_workgroups(n, width, threads):
    u0 = _u0(n, 5)
    steps = 701
    announce("ks ragged", n, width, threads)
    got = run(sw.KS_F64, u0.reshape(1, -1), steps, DT, DX, "swept", width=width, threads=threads)[0]
    assert np.array_equal(got, oracle.ks_f64(u0, steps, DT, DX))


def test_ks_chunked_and_shifted():
    n, w = 4096, 512
    u0 = _u0(n, 9)
    whole = run(sw.KS_F64, u0.reshape(1, -1), 900, DT, DX, "swept", width=w)[0]
    parts = run(sw.KS_F64, u0.reshape(1, -1), 900, DT, DX, "swept", width=w,
                chunks=[1, 299, 77, 523])[0]
    assert np.array_equal(whole, parts)
    k = 37  # not a multiple of W: seams land on other cells
    shifted = run(sw.KS_F64, np.roll(u0, k).reshape(1, -1), 900, DT, DX, "swept", width=w)[0]
    assert np.array_equal(shifted, np.roll(whole, k))


def test_ks_full_size_swept_equals_naive_and_oracle_cones():
    w = wl.KS_PREC
    u0 = wl.initial_state(w)
    announce("fullsize ks swept", w.n, w.steps)
    swept = run(sw.KS_F64, u0.reshape(1, -1), w.steps, w.dt, w.dx, "swept")[0]
    announce("fullsize ks naive")
    naive = run(sw.KS_F64, u0.reshape(1, -1), w.steps, w.dt, w.dx, "naive")[0]
    assert np.array_equal(swept, naive)
    span, reach = 16, 2 * w.steps + 2
    for s0 in (0, w.n // 3 + 5, w.n - 7):
        idx = np.arange(s0 - reach, s0 + span + reach) % w.n
        want = oracle.ks_f64(u0[idx], w.steps, w.dt, w.dx)[reach: reach + span]
        assert np.array_equal(swept[(np.arange(s0, s0 + span)) % w.n], want), s0
    assert np.all(np.isfinite(swept)) and np.max(np.abs(swept)) < 20
