"""Plain CPU oracle of the swept-rule hot path -- test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it.

The numerics live in ``oracle.c`` (binary64 reference of the heat FTCS and
Euler finite-volume schemes of Sec. 4.2 / Fig. 2b, plus the binary32 variant
with binary64 islands).  This module compiles nothing implicitly; it loads
``liboracle.so`` built by :func:`build` and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, no contraction, OpenMP)."""
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
        "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, i32, d, f = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_float
    vp = ctypes.c_void_p
    lib.oracle_heat_f64.argtypes = [vp, i64, i64, d, i32]
    lib.oracle_heat_f32.argtypes = [vp, vp, i64, i64, f, i32]
    lib.oracle_euler_f64.argtypes = [vp, vp, vp, i64, i64, d, i32]
    lib.oracle_euler_f32.argtypes = [vp, vp, vp, vp, vp, vp, i64, i64, f, i32]
    lib.oracle_threads_used.argtypes = [i32]
    lib.oracle_ks_f64.argtypes = [vp, i64, i64, d, d, d, i32]
    for fn in (lib.oracle_heat_f64, lib.oracle_heat_f32, lib.oracle_euler_f64,
               lib.oracle_euler_f32, lib.oracle_threads_used, lib.oracle_ks_f64):
        fn.restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def threads_used(threads: int = 0) -> int:
    return int(_load().oracle_threads_used(int(threads)))


def heat_f64(u0, steps: int, r: float, threads: int = 0) -> np.ndarray:
    """FTCS heat equation, binary64, periodic; returns the state after ``steps``."""
    u = np.array(u0, dtype=np.float64, copy=True, order="C")
    rc = _load().oracle_heat_f64(_ptr(u), u.size, int(steps), float(r), int(threads))
    if rc:
        raise ValueError(f"oracle_heat_f64 failed ({rc})")
    return u


def heat_f32(u0, c0, steps: int, r: float, threads: int = 0):
    """binary32 FTCS with Kahan-compensated update; ``r`` is rounded to binary32 once."""
    u = np.array(u0, dtype=np.float32, copy=True, order="C")
    c = np.array(c0, dtype=np.float32, copy=True, order="C")
    assert u.shape == c.shape
    rc = _load().oracle_heat_f32(_ptr(u), _ptr(c), u.size, int(steps),
                                 float(np.float32(r)), int(threads))
    if rc:
        raise ValueError(f"oracle_heat_f32 failed ({rc})")
    return u, c


def euler_f64(q0, steps: int, lam: float, threads: int = 0) -> np.ndarray:
    """Euler equations, binary64; ``q0`` has shape (3, n) = (rho, m, E)."""
    q = np.array(q0, dtype=np.float64, copy=True, order="C")
    assert q.ndim == 2 and q.shape[0] == 3
    n = q.shape[1]
    rc = _load().oracle_euler_f64(_ptr(q[0]), _ptr(q[1]), _ptr(q[2]), n, int(steps),
                                  float(lam), int(threads))
    if rc:
        raise ValueError(f"oracle_euler_f64 failed ({rc})")
    return q


def euler_f32(q0, c0, steps: int, lam: float, threads: int = 0):
    """binary32 Euler with Kahan-compensated corrector and binary64 islands."""
    q = np.array(q0, dtype=np.float32, copy=True, order="C")
    c = np.array(c0, dtype=np.float32, copy=True, order="C")
    assert q.shape == c.shape and q.shape[0] == 3
    n = q.shape[1]
    rc = _load().oracle_euler_f32(_ptr(q[0]), _ptr(q[1]), _ptr(q[2]), _ptr(c[0]),
                                  _ptr(c[1]), _ptr(c[2]), n, int(steps),
                                  float(np.float32(lam)), int(threads))
    if rc:
        raise ValueError(f"oracle_euler_f32 failed ({rc})")
    return q, c


def ks_coefficients(dt: float, dx: float):
    """(a, b, c) = (dt / (2 dx), dt / dx^2, dt / dx^4), evaluated in binary64 in
    this form; the Kuramoto-Sivashinsky scheme takes them as given."""
    return dt / (2.0 * dx), dt / (dx * dx), dt / ((dx * dx) * (dx * dx))


def ks_f64(u0, steps: int, dt: float, dx: float, threads: int = 0) -> np.ndarray:
    """Kuramoto-Sivashinsky equation, forward Euler / central differences,
    binary64, periodic; returns the state after ``steps``."""
    u = np.array(u0, dtype=np.float64, copy=True, order="C")
    a, b, c = ks_coefficients(dt, dx)
    rc = _load().oracle_ks_f64(_ptr(u), u.size, int(steps), a, b, c, int(threads))
    if rc:
        raise ValueError(f"oracle_ks_f64 failed ({rc})")
    return u
