"""Pins of the Kuramoto-Sivashinsky oracle (u_t + u u_x + u_xx + u_xxxx = 0,
forward Euler, central differences; the scheme is a chosen reading: the
paper names the equation, Sec. 2, but gives no scheme).

* Exact rational brute force from the five-point formulas
      u_xx   ~ (u_{i+1} - 2 u_i + u_{i-1}) / dx^2
      u_xxxx ~ (u_{i+2} - 4 u_{i+1} + 6 u_i - 4 u_{i-1} + u_{i-2}) / dx^4
      (u^2/2)_x ~ (u_{i+1}^2 - u_{i-1}^2) / (4 dx)
  (not the staged form the oracle uses) on tiny grids: agreement to rounding.
* Mirror symmetry: the equation is invariant under x -> -x, u -> -u, and the
  discrete scheme is too, exactly in IEEE arithmetic (every term changes sign
  with sign-symmetric rounding; the outer sums commute).
* Conservation of sum(u) (every difference telescopes) to rounding.
* A small single Fourier mode grows by the linear amplification factor
  G = 1 + 4 b sin^2(theta/2) - 16 c sin^4(theta/2) per step (the advection
  term is second order in the amplitude).
* A constant state is a fixed point, bit for bit.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _brute(u0, steps, dt, dx):
    u = [Fraction(x) for x in u0]
    n = len(u)
    dt, dx = Fraction(dt), Fraction(dx)
    for _ in range(steps):
        new = []
        for i in range(n):
            um2, um1, u0_, up1, up2 = (u[(i + k) % n] for k in (-2, -1, 0, 1, 2))
            uxx = (up1 - 2 * u0_ + um1) / dx ** 2
            uxxxx = (up2 - 4 * up1 + 6 * u0_ - 4 * um1 + um2) / dx ** 4
            adv = (up1 ** 2 - um1 ** 2) / (4 * dx)
            new.append(u0_ - dt * (adv + uxx + uxxxx))
        u = new
    return np.array([float(x) for x in u])


@pytest.mark.parametrize("n,steps,dt,dx,seed", [(10, 3, 1 / 16, 1.0, 1), (12, 4, 1 / 32, 0.5, 2),
                                                 (7, 5, 0.01, 1.25, 3)])
def test_brute_force_rational(n, steps, dt, dx, seed):
    rng = np.random.default_rng(seed)
    u0 = np.round(rng.uniform(-2, 2, n) * 64) / 64  # dyadic: exact in binary64
    want = _brute(u0, steps, dt, dx)
    got = oracle.ks_f64(u0, steps, dt, dx)
    scale = max(1.0, float(np.max(np.abs(want))))
    assert np.max(np.abs(got - want)) <= 1e-13 * scale, (got, want)


def test_brute_force_catches_a_wrong_sign():
    """The brute-force pin is sharp: flipping the sign of the advection term
    in the reference changes the result far beyond rounding."""
    u0 = np.array([0.5, 1.25, -0.75, 0.25, 2.0, -1.5, 0.0, 1.0, -0.25, 0.75])
    good = _brute(u0, 2, 1 / 16, 1.0)
    got = oracle.ks_f64(u0, 2, 1 / 16, 1.0)
    mirror = -_brute(-u0, 2, 1 / 16, 1.0)  # = the scheme with u u_x negated
    assert np.max(np.abs(got - good)) < 1e-13
    assert np.max(np.abs(mirror - good)) > 1e-3


@pytest.mark.parametrize("n,steps", [(64, 200), (1000, 137)])
def test_mirror_symmetry_exact(n, steps):
    rng = np.random.default_rng(n)
    x = np.arange(n) / n
    u0 = sum(rng.standard_normal() * np.sin(2 * np.pi * k * x + rng.uniform(0, 6))
             for k in (1, 2, 3, 5, 8))
    a = oracle.ks_f64(u0, steps, 0.05, 1.0)
    b = oracle.ks_f64(-u0[::-1], steps, 0.05, 1.0)
    assert np.array_equal(b, -a[::-1])


def test_conservation_of_the_sum():
    n, steps = 512, 2000
    rng = np.random.default_rng(7)
    u0 = rng.uniform(-1, 1, n)
    u = oracle.ks_f64(u0, steps, 0.05, 1.0)
    drift = abs(np.sum(u, dtype=np.float64) - np.sum(u0, dtype=np.float64))
    import math
    drift = abs(math.fsum(u) - math.fsum(u0))
    assert drift <= 4 * steps * n * np.finfo(float).eps * max(1.0, np.max(np.abs(u)))
    assert np.max(np.abs(u)) < 10  # bounded on the attractor


@pytest.mark.parametrize("k", [1, 3, 7, 20])
def test_linear_growth_of_a_small_mode(k):
    n, steps, dt, dx, eps = 128, 60, 0.05, 1.0, 1e-9
    a, b, c = oracle.ks_coefficients(dt, dx)
    theta = 2 * np.pi * k / n
    g = 1 + 4 * b * np.sin(theta / 2) ** 2 - 16 * c * np.sin(theta / 2) ** 4
    j = np.arange(n)
    u0 = eps * np.sin(theta * j)
    got = oracle.ks_f64(u0, steps, dt, dx)
    want = eps * g ** steps * np.sin(theta * j)
    assert np.max(np.abs(got - want)) <= 1e-6 * eps * max(1.0, g ** steps)


def test_constant_state_is_a_fixed_point():
    u0 = np.full(33, 0.8125)
    assert np.array_equal(oracle.ks_f64(u0, 50, 0.05, 1.0), u0)
