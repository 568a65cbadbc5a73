"""GPU pin of the rounded-to-nearest sequences of the Euler kernels
(paper_1811_08282_amd/csrc/rn_ops.h): the clamp form of the limiter, the
square root that skips the compiler's rescaling on [2^-767, +inf), and two
quotients sharing one refined reciprocal -- against numpy's IEEE limiter
definition, square root and division, bit for bit (any NaN for a NaN), on
random operands over the whole binary64 range, zeros, infinities, NaNs and
values at the 2^-767 threshold.

The helper kernel is tests/rn_check.hip, built into tests/librn_check.so by
the build step.
"""
import ctypes
import os

import numpy as np
import pytest

import paper_1811_08282_amd as sw  # noqa: F401  (loads torch before any HIP library)
from gpu_util import announce

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librn_check.so")


def _lib():
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB)
    lib.rn_check.restype = ctypes.c_int
    lib.rn_check.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64]
    return lib


def _random_doubles(rng, n):
    """Random signs, exponents over the whole range (denormals included) and
    mantissas, plus a share of zeros, infinities, NaNs and ones."""
    bits = (rng.integers(0, 1 << 52, n, dtype=np.uint64)
            | (rng.integers(0, 2047, n, dtype=np.uint64) << np.uint64(52))
            | (rng.integers(0, 2, n, dtype=np.uint64) << np.uint64(63)))
    x = bits.view(np.float64)
    moderate = rng.random(n) < 0.5
    x[moderate] = (rng.choice([-1.0, 1.0], moderate.sum())
                   * np.exp2(rng.uniform(-60, 60, moderate.sum())))
    special = rng.integers(0, 40, n)
    for k, v in enumerate((0.0, -0.0, np.inf, -np.inf, np.nan, 1.0)):
        x[special == k] = v
    return x


def _in_range_doubles(rng, n):
    """Positive values in [2^-767, 2^1023): whole waves of them take the
    square root's short path; the threshold itself and its neighbours too."""
    e = rng.uniform(-767, 1023, n)
    x = np.exp2(e) * rng.uniform(1.0, 2.0, n)
    x = np.minimum(x, np.finfo(np.float64).max)
    x[:64] = 2.0 ** -767
    x[64:128] = np.nextafter(2.0 ** -767, np.inf)
    return x


def _same(got, want):
    both_nan = np.isnan(got) & np.isnan(want)
    return both_nan | (got.view(np.int64) == want.view(np.int64))


@pytest.mark.gpu
def test_rn_ops_equal_ieee_operations():
    import torch
    lib = _lib()
    rng = np.random.default_rng(20261203)
    n_mixed, n_range = 1 << 20, 1 << 20
    a = np.concatenate([_random_doubles(rng, n_mixed), _in_range_doubles(rng, n_range)])
    c = np.concatenate([_random_doubles(rng, n_mixed), _in_range_doubles(rng, n_range)])
    d = np.concatenate([_random_doubles(rng, n_mixed), _random_doubles(rng, n_range)])
    # a few divisors shared with special numerators and the other way round
    d[:16] = [0.0, -0.0, np.inf, np.nan, 2.0 ** -1074, 2.0 ** 1023, -3.0, 1.0,
              1e-300, 1e300, 2.0 ** -1022, 7.0, -0.0, 0.0, 5e-324, 3.0]
    n = a.size
    announce(f"rn ops: {n} operands")
    da, dc, dd = (torch.from_numpy(v).cuda() for v in (a, c, d))
    out = torch.empty(6 * n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    assert lib.rn_check(da.data_ptr(), dc.data_ptr(), dd.data_ptr(), out.data_ptr(), n) == 0
    o = out.cpu().numpy().reshape(n, 6)
    with np.errstate(all="ignore"):
        lim = np.where(a > 0.0, np.minimum(a, 1.0), 0.0)
        want = [lim, np.sqrt(a), a / d, c / d, np.sqrt(a), np.sqrt(c)]
    names = ["limiter", "sqrt", "first quotient", "second quotient", "sqrt pair (a)",
             "sqrt pair (c)"]
    for k, (name, w) in enumerate(zip(names, want)):
        ok = _same(o[:, k], w)
        bad = np.flatnonzero(~ok)
        assert bad.size == 0, (
            f"{name}: {bad.size} mismatches, first at {bad[0]}: "
            f"a={a[bad[0]]!r} c={c[bad[0]]!r} d={d[bad[0]]!r} got {o[bad[0], k]!r} "
            f"want {w[bad[0]]!r}")
    # the limiter maps -0 and NaN to +0 exactly
    assert (o[:, 0].view(np.int64)[(a == 0) | np.isnan(a)] == 0).all()
