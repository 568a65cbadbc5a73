"""Seeded synthetic inputs for the swept-rule workloads.

This module holds the initial-condition generators shared by the tests, the
benchmark and the oracle checks.  It contains none of the schemes'
arithmetic: it only builds initial states and problem lists.

The paper's own initial conditions are not given in the text (the schemes are
deferred to the authors' earlier article, Sec. 4.2), so synthetic inputs of
the paper's shapes stand in for them:

* heat  -- a sum of ``n_modes`` sine modes with N(0, 1) amplitudes and
  distinct integer wavenumbers; the grid is periodic so every mode is exact.
* euler -- a periodic tiling of the Sod shock-tube states
  (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1), i.e. conserved
  (rho, m, E) = (1, 0, 2.5) | (0.125, 0, 0.25) with gamma = 1.4.
* batch -- many independent problems with log-uniform lengths.
* ks    -- the Kuramoto-Sivashinsky equation (no workload in the paper): the
  heat recipe's random modes scaled by 0.1, dt = 0.02, dx = 1
  (a = 0.01, b = c = 0.02); the modes lie in the band the equation
  amplifies, and the solution saturates at |u| of about 4 (forward Euler on
  the central advection term stays stable there; at dt = 0.05 or with
  unscaled modes it does not).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SOD_LEFT = (1.0, 0.0, 2.5)      # rho, m, E  for (rho, u, p) = (1, 0, 1)
SOD_RIGHT = (0.125, 0.0, 0.25)  # rho, m, E  for (rho, u, p) = (0.125, 0, 0.1)


def distinct_wavenumbers(rng: np.random.Generator, count: int, kmin: int, kmax: int,
                         log_uniform: bool) -> np.ndarray:
    """Draw ``count`` distinct integers in [kmin, kmax], uniform or log-uniform."""
    if kmax - kmin + 1 < count:
        raise ValueError("not enough distinct wavenumbers in range")
    out: list[int] = []
    while len(out) < count:
        if log_uniform:
            k = int(math.floor(math.exp(rng.uniform(math.log(kmin), math.log(kmax + 1)))))
        else:
            k = int(rng.integers(kmin, kmax + 1))
        k = min(max(k, kmin), kmax)
        if k not in out:
            out.append(k)
    return np.array(out, dtype=np.int64)


def sine_modes(n: int, ks: np.ndarray, amps: np.ndarray) -> np.ndarray:
    """u_j = sum_m a_m sin(2 pi k_m j / n), phases reduced exactly in integers."""
    j = np.arange(n, dtype=np.int64)
    u = np.zeros(n, dtype=np.float64)
    for k, a in zip(ks.tolist(), amps.tolist()):
        t = (int(k) * j) % n
        u += a * np.sin((2.0 * np.pi / n) * t.astype(np.float64))
    return u


def heat_ic(n: int, seed: int, n_modes: int = 8, kmax: int | None = None,
            log_uniform: bool = True) -> np.ndarray:
    """Random-mode heat initial condition (binary64).

    ``kmax`` defaults to n // 16.  Wavenumbers are drawn first, then the
    amplitudes, from ``numpy.random.default_rng(seed)``.
    """
    rng = np.random.default_rng(seed)
    if kmax is None:
        kmax = max(n // 16, n_modes)
    ks = distinct_wavenumbers(rng, n_modes, 1, kmax, log_uniform)
    amps = rng.standard_normal(n_modes)
    return sine_modes(n, ks, amps)


def sod_tiled(n: int, tile: int) -> np.ndarray:
    """Conserved Sod states tiled with period ``tile``; shape (3, n), binary64.

    Cell j is in the left state when (j mod tile) < tile / 2.
    """
    if tile <= 0 or tile % 2:
        raise ValueError("tile must be a positive even number")
    j = np.arange(n, dtype=np.int64)
    left = (j % tile) < (tile // 2)
    q = np.empty((3, n), dtype=np.float64)
    for k in range(3):
        q[k] = np.where(left, SOD_LEFT[k], SOD_RIGHT[k])
    return q


# --------------------------------------------------------------------------
# named workloads (sizes of the benchmark configurations)
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    eq: str          # "heat" | "euler"
    n: int
    steps: int
    dt: float
    dx: float
    seed: int | None
    tile: int | None = None


HEAT_SMALL = Workload("heat_f64_n1024_s1000", "heat", 1024, 1000, 0.25, 1.0, 1)
HEAT_LARGE = Workload("heat_f64_n4194304_s20000", "heat", 1 << 22, 20000, 0.25, 1.0, 2)
EULER_LARGE = Workload("euler_f64_n4194304_s10000", "euler", 1 << 22, 10000, 0.1, 1.0, None, 1 << 14)
HEAT_PREC = Workload("heat_n16777216_s20000", "heat", 1 << 24, 20000, 0.25, 1.0, 4)
EULER_PREC = Workload("euler_n16777216_s20000", "euler", 1 << 24, 20000, 0.1, 1.0, None, 1 << 14)
KS_PREC = Workload("ks_n16777216_s20000", "ks", 1 << 24, 20000, 0.02, 1.0, 6)


def initial_state(w: Workload) -> np.ndarray:
    """binary64 initial state of a workload: (n,) for heat and
    Kuramoto-Sivashinsky, (3, n) for Euler."""
    if w.eq == "ks":
        return ks_ic(w.n, w.seed)
    if w.eq == "heat":
        if w.n == 1024:
            return heat_ic(w.n, w.seed, kmax=32, log_uniform=False)
        return heat_ic(w.n, w.seed)
    return sod_tiled(w.n, w.tile)


def ks_ic(n: int, seed: int) -> np.ndarray:
    """Kuramoto-Sivashinsky initial condition: the heat modes scaled by 0.1."""
    return 0.1 * heat_ic(n, seed)


@dataclass(frozen=True)
class BatchProblem:
    index: int
    eq: str
    n: int


def batch_problems(count: int = 4096, seed: int = 5, lo: float = 10.0, hi: float = 18.0,
                   quantum: int = 256, min_quanta: int = 4) -> list[BatchProblem]:
    """Problem list of the batched workload.

    u_p ~ U[lo, hi] from ``default_rng(seed)``;
    L_p = quantum * max(min_quanta, round(2**u_p / quantum)); even p -> heat,
    odd p -> Euler.
    """
    rng = np.random.default_rng(seed)
    us = rng.uniform(lo, hi, size=count)
    out = []
    for p, u in enumerate(us.tolist()):
        n = quantum * max(min_quanta, int(round(2.0 ** u / quantum)))
        out.append(BatchProblem(p, "heat" if p % 2 == 0 else "euler", n))
    return out


def batch_ic(prob: BatchProblem, base_seed: int = 5) -> np.ndarray:
    """Initial state of one batch problem (binary64)."""
    if prob.eq == "heat":
        return heat_ic(prob.n, base_seed + prob.index)
    return sod_tiled(prob.n, prob.n)
