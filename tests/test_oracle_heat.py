"""Pins of the heat-equation oracle against what the mathematics fixes.

The scheme is FTCS (Sec. 4.2 of the paper); none of these checks re-types it:
they compare with the binomial closed form, the Fourier amplification factor,
exact rational arithmetic, and invariants (mirror / shift symmetry,
conservation, maximum principle).
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle


def _binomial_profile(n_cells, center, steps):
    """Exact impulse response of FTCS at r = 1/4 on a periodic grid.

    At r = 1/4 one step is convolution with [1, 2, 1] / 4 = ([1, 1] / 2)^2, so
    after n steps the kernel is C(2n, n + d) / 4^n, summed over periodic images.
    """
    out = [Fraction(0)] * n_cells
    for d in range(-steps, steps + 1):
        out[(center + d) % n_cells] += Fraction(math.comb(2 * steps, steps + d), 4 ** steps)
    return out


@pytest.mark.parametrize("n_cells,center,steps", [(128, 60, 1), (128, 3, 7), (128, 127, 26),
                                                   (64, 0, 26), (16, 5, 20), (9, 4, 13)])
def test_impulse_matches_binomial_exactly(n_cells, center, steps):
    u = np.zeros(n_cells)
    u[center] = 1.0
    got = oracle.heat_f64(u, steps, 0.25)
    want = np.array([float(x) for x in _binomial_profile(n_cells, center, steps)])
    # every value is a dyadic rational with at most 52 significant bits
    assert np.array_equal(got, want)


def test_impulse_f32_exact_and_zero_compensation():
    n, steps = 64, 11  # values are multiples of 4^-11 = 2^-22: exact in binary32
    u = np.zeros(n, np.float32)
    u[17] = 1.0
    got, c = oracle.heat_f32(u, np.zeros(n, np.float32), steps, 0.25)
    want = np.array([float(x) for x in _binomial_profile(n, 17, steps)], np.float32)
    assert np.array_equal(got, want)
    assert not np.any(c)


@pytest.mark.parametrize("r", [0.25, 0.4, 0.1])
@pytest.mark.parametrize("k", [1, 5, 37])
def test_fourier_mode_amplification(r, k):
    n, steps = 256, 400
    j = np.arange(n)
    u0 = np.sin(2 * np.pi * k * j / n) + 0.5 * np.cos(2 * np.pi * k * j / n)
    got = oracle.heat_f64(u0, steps, r)
    mpmath.mp.dps = 40
    g = 1 - 4 * mpmath.mpf(r) * mpmath.sin(mpmath.pi * k / n) ** 2
    amp = float(g ** steps)
    want = amp * u0
    # rounding accumulates ~steps * eps; the closed form itself is exact
    assert np.max(np.abs(got - want)) <= 1e-12 * steps * np.max(np.abs(u0))


def test_rational_brute_force_exact_and_rounding_bound():
    rng = np.random.default_rng(11)
    for n in (8, 11, 16):
        u0 = rng.integers(-64, 64, size=n) / 64.0  # dyadic
        for r in (Fraction(1, 4), Fraction(3, 10)):
            cur = [Fraction(x) for x in u0]
            for _ in range(6):
                cur = [cur[i] + r * (cur[(i + 1) % n] + cur[i - 1] - 2 * cur[i]) for i in range(n)]
            got = oracle.heat_f64(u0, 6, float(r))
            want = np.array([float(x) for x in cur])
            if r.denominator == 4:
                assert np.array_equal(got, want)
            else:
                assert np.max(np.abs(got - want)) < 1e-14


def test_mirror_and_shift_symmetry_bitexact():
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal(300)
    base = oracle.heat_f64(u0, 137, 0.3)
    mir = oracle.heat_f64(u0[::-1], 137, 0.3)
    assert np.array_equal(mir[::-1], base)
    for s in (1, 77, 299):
        sh = oracle.heat_f64(np.roll(u0, s), 137, 0.3)
        assert np.array_equal(sh, np.roll(base, s))


def test_conservation_and_maximum_principle():
    rng = np.random.default_rng(4)
    u0 = rng.uniform(-1.0, 2.0, 500)
    steps = 2000
    got = oracle.heat_f64(u0, steps, 0.45)
    drift = abs(math.fsum(got) - math.fsum(u0))
    assert drift <= 4 * steps * u0.size * np.finfo(float).eps * np.max(np.abs(u0))
    assert got.min() >= u0.min() - 1e-12 and got.max() <= u0.max() + 1e-12


def test_f32_kahan_tracks_f64():
    n, steps = 4096, 20000
    u64 = np.sin(2 * np.pi * 3 * np.arange(n) / n) + 0.25 * np.sin(2 * np.pi * 40 * np.arange(n) / n)
    u32 = u64.astype(np.float32)
    ref = oracle.heat_f64(u32.astype(np.float64), steps, 0.25)
    got, _ = oracle.heat_f32(u32, np.zeros(n, np.float32), steps, 0.25)
    rel = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert rel < 1e-6


def test_thread_count_does_not_change_result():
    u0 = np.random.default_rng(9).standard_normal(10007)
    a = oracle.heat_f64(u0, 50, 0.25, threads=1)
    b = oracle.heat_f64(u0, 50, 0.25, threads=4)
    assert np.array_equal(a, b)
