"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, and
swept against naive, element by element on seeded inputs.

Bars (floating point, written here):
* binary64: swept == naive bit for bit; both == oracle bit for bit (the
  same IEEE operation sequence, no contraction, correctly rounded divide and
  square root); the stated bound is 1e-12 relative and the tests also assert
  exact equality.
* binary32: swept == naive bit for bit; both == the binary32 oracle bit for
  bit; error against the binary64 oracle stated per test.
"""
import numpy as np
import pytest

import oracle
import paper_1811_08282_amd as sw
from paper_1811_08282_amd.workloads import heat_ic, sod_tiled
from gpu_util import announce, pack, rel_inf, run

pytestmark = pytest.mark.gpu


def _smooth_euler(n, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(n) / n
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * 3 * x + rng.uniform(0, 6))
    u = 0.3 * np.cos(2 * np.pi * 5 * x)
    p = 1.0 + 0.25 * np.sin(2 * np.pi * 7 * x + 1.0)
    return np.array([rho, rho * u, p / 0.4 + 0.5 * rho * u * u])


# ---- heat, binary64 ----------------------------------------------------------

def test_heat_f64_small_config_naive_and_swept_equal_oracle():
    n, steps = 1024, 1000
    u0 = heat_ic(n, 1, kmax=32, log_uniform=False)
    want = oracle.heat_f64(u0, steps, 0.25)
    announce("heat_f64 n=1024 steps=1000 naive")
    naive = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), steps, 0.25, 1.0, "naive")[0]
    announce("heat_f64 n=1024 steps=1000 swept W=64")
    swept = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), steps, 0.25, 1.0, "swept", width=64)[0]
    assert rel_inf(naive, want) <= 1e-12 and np.array_equal(naive, want)
    assert np.array_equal(swept, naive)


@pytest.mark.parametrize("width", [2, 4, 8, 16, 32, 64, 128, 256, 512])
def test_heat_f64_swept_every_width(width):
    n = 1024
    u0 = heat_ic(n, 3)
    rng = np.random.default_rng(width)
    for steps in sorted({1, width // 2, width // 2 + 1, 3 * width + 5, int(rng.integers(1, 700))}):
        announce("heat_f64 swept W", width, "steps", steps)
        got = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), steps, 0.3, 1.0, "swept", width=width)[0]
        want = oracle.heat_f64(u0, steps, 0.3)
        assert np.array_equal(got, want), (width, steps, rel_inf(got, want))


# The heat level sweep runs in register blocks of four levels: rows of 62
# lanes x 4 cells, a row aligned to each window edge (the right one stored
# mirrored), LDS only between blocks, and a level-by-level fallback for
# narrow windows.  Cases: several rows per wave, odd W/2 (odd level parity
# at the phase starts), 64- to 512-thread workgroups, flat cuts at a step
# count that is not a multiple of W/2, and W = 4096 in 256 threads, where
# the widest windows need more rows than four waves hold and fall back.
@pytest.mark.parametrize("eq", [sw.HEAT_F64, sw.HEAT_F32])
@pytest.mark.parametrize("n,width,threads,steps", [
    (3 * 2048, 2048, 256, 2 * 1024 + 517), (4 * 1030, 1030, 128, 1500),
    (2 * 4096, 4096, 512, 4096 + 33), (2 * 4096, 4096, 256, 2100), (2 * 518, 518, 64, 777),
    (8 * 1024, 1024, 256, 3001)])
def test_heat_register_blocked_sweep(eq, n, width, threads, steps):
    u0 = heat_ic(n, width + steps)
    announce("heat register-blocked sweep", eq, n, width, threads, steps)
    got = run(eq, pack(eq, u0), steps, 0.25, 1.0, "swept", width=width, threads=threads)
    if eq == sw.HEAT_F64:
        want = oracle.heat_f64(u0, steps, 0.25).reshape(1, -1)
    else:
        u32 = u0.astype(np.float32)
        want = np.stack(oracle.heat_f32(u32, np.zeros_like(u32), steps, 0.25))
    assert np.array_equal(got, want), (eq, n, width, threads, steps)


@pytest.mark.parametrize("n,width", [(1000, 40), (1000, 250), (6, 2), (4098, 2), (3 * 2048, 1024),
                                     (2 * 8192, 8192)])
def test_heat_f64_ragged_and_extreme_shapes(n, width):
    u0 = np.random.default_rng(n).standard_normal(n)
    steps = 777
    announce("heat_f64 shape n", n, "W", width)
    got = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), steps, 0.2, 1.0, "swept", width=width)[0]
    naive = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), steps, 0.2, 1.0, "naive")[0]
    want = oracle.heat_f64(u0, steps, 0.2)
    assert np.array_equal(naive, want)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("eq", [sw.HEAT_F64, sw.HEAT_F32])
def test_heat_single_step_all_widths(eq):
    """One heat step is a single phase that cannot write the state it reads."""
    n = 2048
    u0 = heat_ic(n, 12)
    want = run(eq, pack(eq, u0), 1, 0.3, 1.0, "naive")
    for width in (2, 64, 256, 1024):
        announce("heat single step eq", eq, "W", width)
        got = run(eq, pack(eq, u0), 1, 0.3, 1.0, "swept", width=width)
        assert np.array_equal(got, want)


def test_heat_f64_naive_odd_sizes_and_default_width():
    for n in (3, 5, 257):
        u0 = np.random.default_rng(n).standard_normal(n)
        announce("heat_f64 naive n", n)
        got = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), 31, 0.25, 1.0, "naive")[0]
        assert np.array_equal(got, oracle.heat_f64(u0, 31, 0.25))
    u0 = heat_ic(1 << 14, 8)
    announce("heat_f64 swept default width n=16384")
    got = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), 600, 0.25, 1.0, "swept")[0]
    assert np.array_equal(got, oracle.heat_f64(u0, 600, 0.25))


def test_heat_f64_chunked_shift_and_determinism():
    n, w = 2048, 128
    u0 = heat_ic(n, 5)
    announce("heat_f64 chunked")
    one = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), 500, 0.25, 1.0, "swept", width=w)[0]
    parts = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), 500, 0.25, 1.0, "swept", width=w,
                chunks=[1, 63, 200, 236])[0]
    assert np.array_equal(one, parts)
    announce("heat_f64 shift")
    sh = run(sw.HEAT_F64, pack(sw.HEAT_F64, np.roll(u0, 37)), 500, 0.25, 1.0, "swept", width=w)[0]
    assert np.array_equal(sh, np.roll(one, 37))
    again = run(sw.HEAT_F64, pack(sw.HEAT_F64, u0), 500, 0.25, 1.0, "swept", width=w)[0]
    assert np.array_equal(again, one)


# ---- heat, binary32 + Kahan ----------------------------------------------------

@pytest.mark.parametrize("width", [2, 64, 256, 1024])
def test_heat_f32_matches_f32_oracle_bitexact(width):
    n, steps = 4096, 3000
    u0 = heat_ic(n, 6)
    u32 = u0.astype(np.float32)
    want_u, want_c = oracle.heat_f32(u32, np.zeros(n, np.float32), steps, 0.25)
    announce("heat_f32 swept W", width)
    sw_state = run(sw.HEAT_F32, pack(sw.HEAT_F32, u0), steps, 0.25, 1.0, "swept", width=width)
    announce("heat_f32 naive")
    nv_state = run(sw.HEAT_F32, pack(sw.HEAT_F32, u0), steps, 0.25, 1.0, "naive")
    assert np.array_equal(nv_state[0], want_u) and np.array_equal(nv_state[1], want_c)
    assert np.array_equal(sw_state, nv_state)
    ref64 = oracle.heat_f64(u32.astype(np.float64), steps, 0.25)
    assert rel_inf(sw_state[0], ref64) < 1e-6


# ---- Euler, binary64 ----------------------------------------------------------

@pytest.mark.parametrize("kind", ["sod", "smooth"])
def test_euler_f64_naive_equals_oracle(kind):
    n, steps = 2048, 300
    q0 = sod_tiled(n, 512) if kind == "sod" else _smooth_euler(n, 1)
    announce("euler_f64 naive", kind)
    got = run(sw.EULER_F64, pack(sw.EULER_F64, q0), steps, 0.1, 1.0, "naive")
    want = oracle.euler_f64(q0, steps, 0.1)
    assert rel_inf(got, want) <= 1e-12
    assert np.array_equal(got, want)


@pytest.mark.parametrize("width", [2, 8, 64, 128, 256, 512, 1024])
def test_euler_f64_swept_every_width(width):
    n = 2048
    q0 = sod_tiled(n, 512)
    q0[1] += 0.05 * q0[0]  # a drift makes the tiles' work asymmetric
    rng = np.random.default_rng(width)
    want_cache = {}
    for steps in sorted({1, max(1, width // 8), width // 8 + 1, int(rng.integers(1, 300))}):
        announce("euler_f64 swept W", width, "steps", steps)
        got = run(sw.EULER_F64, pack(sw.EULER_F64, q0), steps, 0.1, 1.0, "swept", width=width)
        want = want_cache.setdefault(steps, oracle.euler_f64(q0, steps, 0.1))
        assert np.array_equal(got, want), (width, steps, rel_inf(got, want))


def test_euler_f64_chunked_and_shift():
    n, w = 1024, 128
    q0 = _smooth_euler(n, 2)
    announce("euler_f64 chunked")
    one = run(sw.EULER_F64, pack(sw.EULER_F64, q0), 150, 0.1, 1.0, "swept", width=w)
    parts = run(sw.EULER_F64, pack(sw.EULER_F64, q0), 150, 0.1, 1.0, "swept", width=w,
                chunks=[7, 50, 93])
    assert np.array_equal(one, parts)
    announce("euler_f64 shift")
    sh = run(sw.EULER_F64, pack(sw.EULER_F64, np.roll(q0, 45, axis=1)), 150, 0.1, 1.0, "swept",
             width=w)
    assert np.array_equal(sh, np.roll(one, 45, axis=1))


# ---- Euler, binary32 -------------------------------------------------------------

@pytest.mark.parametrize("width", [2, 64, 256, 1024])
def test_euler_f32_matches_f32_oracle_bitexact(width):
    n, steps = 2048, 400
    q0 = sod_tiled(n, 1024)
    q32 = q0.astype(np.float32)
    want_q, want_c = oracle.euler_f32(q32, np.zeros_like(q32), steps, 0.1)
    announce("euler_f32 swept W", width)
    swp = run(sw.EULER_F32, pack(sw.EULER_F32, q0), steps, 0.1, 1.0, "swept", width=width)
    announce("euler_f32 naive")
    nv = run(sw.EULER_F32, pack(sw.EULER_F32, q0), steps, 0.1, 1.0, "naive")
    assert np.array_equal(nv[:3], want_q) and np.array_equal(nv[3:], want_c)
    assert np.array_equal(swp, nv)
    ref64 = oracle.euler_f64(q32.astype(np.float64), steps, 0.1)
    rel1 = np.abs(swp[:3] - ref64).sum(axis=1) / np.abs(ref64).sum(axis=1)
    assert rel1[0] < 1e-3 and rel1[2] < 1e-3


# ---- Euler, flattened layout (two five-point sub-steps per step) ------------------

@pytest.mark.parametrize("width", [4, 8, 64, 256, 1024])
def test_euler_flat_f64_equals_lengthened_and_oracle(width):
    n = 2048
    q0 = sod_tiled(n, 512)
    q0[1] += 0.05 * q0[0]
    rng = np.random.default_rng(100 + width)
    for steps in sorted({1, 2, max(1, width // 4), int(rng.integers(1, 300))}):
        want = oracle.euler_f64(q0, steps, 0.1)
        announce("euler_f64_flat swept W", width, "steps", steps)
        got = run(sw.EULER_F64_FLAT, pack(sw.EULER_F64, q0), steps, 0.1, 1.0, "swept", width=width)
        assert np.array_equal(got, want), (width, steps, rel_inf(got, want))
    announce("euler_f64_flat naive")
    naive = run(sw.EULER_F64_FLAT, pack(sw.EULER_F64, q0), steps, 0.1, 1.0, "naive")
    assert np.array_equal(naive, want)


def test_euler_flat_f64_ragged_chunked_shift():
    n, w = 1000, 40
    q0 = _smooth_euler(n, 3)
    announce("euler_f64_flat ragged")
    one = run(sw.EULER_F64_FLAT, pack(sw.EULER_F64, q0), 111, 0.1, 1.0, "swept", width=w)
    assert np.array_equal(one, oracle.euler_f64(q0, 111, 0.1))
    parts = run(sw.EULER_F64_FLAT, pack(sw.EULER_F64, q0), 111, 0.1, 1.0, "swept", width=w,
                chunks=[1, 10, 100])
    assert np.array_equal(parts, one)
    sh = run(sw.EULER_F64_FLAT, pack(sw.EULER_F64, np.roll(q0, 13, axis=1)), 111, 0.1, 1.0,
             "swept", width=w)
    assert np.array_equal(sh, np.roll(one, 13, axis=1))


@pytest.mark.parametrize("width", [4, 64, 512])
def test_euler_flat_f32_matches_f32_oracle_bitexact(width):
    n, steps = 2048, 300
    q0 = sod_tiled(n, 1024)
    q32 = q0.astype(np.float32)
    want_q, want_c = oracle.euler_f32(q32, np.zeros_like(q32), steps, 0.1)
    announce("euler_f32_flat swept W", width)
    swp = run(sw.EULER_F32_FLAT, pack(sw.EULER_F32, q0), steps, 0.1, 1.0, "swept", width=width)
    announce("euler_f32_flat naive")
    nv = run(sw.EULER_F32_FLAT, pack(sw.EULER_F32, q0), steps, 0.1, 1.0, "naive")
    assert np.array_equal(nv[:3], want_q) and np.array_equal(nv[3:], want_c)
    assert np.array_equal(swp, nv)


@pytest.mark.parametrize("eq", [sw.HEAT_F64, sw.HEAT_F32, sw.EULER_F64, sw.EULER_F32,
                                sw.EULER_F64_FLAT, sw.EULER_F32_FLAT])
def test_widest_tile_of_every_equation(eq):
    """The largest width the LDS allows (close to the 160 KiB of one CU for
    Euler), two tiles, enough steps for at least three phases: swept equals
    the classic path and the oracle of the same precision bit for bit."""
    w = sw.sw_max_width(eq)
    n = 2 * w
    half = w // (2 * sw.radius(eq))
    steps = (2 * half + 2 + sw.substeps(eq) - 1) // sw.substeps(eq) + 3
    announce("widest tile", eq, w, steps)
    if eq in (sw.HEAT_F64, sw.HEAT_F32):
        q0 = heat_ic(n, 12)
        dt, dx = 0.25, 1.0
    else:
        q0 = sod_tiled(n, n)
        dt, dx = 0.1, 1.0
    layout = {sw.EULER_F64_FLAT: sw.EULER_F64, sw.EULER_F32_FLAT: sw.EULER_F32}.get(eq, eq)
    host = pack(layout, q0)
    swept = run(eq, host, steps, dt, dx, "swept", width=w)
    naive = run(eq, host, steps, dt, dx, "naive")
    assert np.array_equal(swept, naive)
    if eq == sw.HEAT_F64:
        want = oracle.heat_f64(host[0], steps, dt / dx ** 2).reshape(1, -1)
    elif eq == sw.HEAT_F32:
        want = np.stack(oracle.heat_f32(host[0], host[1], steps, dt / dx ** 2))
    elif eq in (sw.EULER_F64, sw.EULER_F64_FLAT):
        want = oracle.euler_f64(host, steps, dt / dx)
    else:
        want = np.concatenate(oracle.euler_f32(host[:3], host[3:], steps, dt / dx))
    assert np.array_equal(swept, want)


@pytest.mark.parametrize("eq", [sw.HEAT_F64, sw.HEAT_F32, sw.EULER_F64, sw.EULER_F32,
                                sw.EULER_F64_FLAT, sw.EULER_F32_FLAT])
def test_512_thread_workgroups_every_equation(eq):
    """Eight-wave workgroups (the default launch of Euler tiles of 1024 cells
    and more) at compile-time widths (1024, 2048) and a run-time one (1536):
    bit-identical to the oracle of the same precision for step counts that
    end inside the first, second and later phases."""
    n = 3 * 2048
    if eq in (sw.HEAT_F64, sw.HEAT_F32):
        q0 = heat_ic(n, 31)
        dt, dx = 0.25, 1.0
    else:
        q0 = sod_tiled(n, 1024)
        q0[1] += 0.05 * q0[0]
        dt, dx = 0.1, 1.0
    layout = {sw.EULER_F64_FLAT: sw.EULER_F64, sw.EULER_F32_FLAT: sw.EULER_F32}.get(eq, eq)
    host = pack(layout, q0)
    for w in (1024, 1536, 2048):
        half_steps = (w // (2 * sw.radius(eq))) // sw.substeps(eq)
        for steps in (1, half_steps, half_steps + 1, 3 * half_steps + 7):
            announce("512 threads eq", eq, "W", w, "steps", steps)
            got = run(eq, host, steps, dt, dx, "swept", width=w, threads=512)
            if eq == sw.HEAT_F64:
                want = oracle.heat_f64(host[0], steps, dt / dx ** 2).reshape(1, -1)
            elif eq == sw.HEAT_F32:
                want = np.stack(oracle.heat_f32(host[0], host[1], steps, dt / dx ** 2))
            elif eq in (sw.EULER_F64, sw.EULER_F64_FLAT):
                want = oracle.euler_f64(host, steps, dt / dx)
            else:
                want = np.concatenate(oracle.euler_f32(host[:3], host[3:], steps, dt / dx))
            assert np.array_equal(got, want), (eq, w, steps)
