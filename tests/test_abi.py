"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/swept.h, sizes its buffers as documented, and rejects
invalid arguments on the host before any HIP call."""
import ctypes
import math
import os
import re

import pytest

import paper_1811_08282_amd as sw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swept.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_library_exports_every_declared_function():
    lib = sw.load()
    names = _declared_functions()
    assert "swept_solve" in names and "naive_solve" in names and len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name


def test_state_and_workspace_sizes():
    n = 1 << 10
    assert sw.sw_state_bytes(sw.HEAT_F64, n) == 8 * n
    assert sw.sw_state_bytes(sw.HEAT_F32, n) == 8 * n
    assert sw.sw_state_bytes(sw.EULER_F64, n) == 24 * n
    assert sw.sw_state_bytes(sw.EULER_F32, n) == 24 * n
    assert sw.sw_state_bytes(7, n) == 0
    assert sw.sw_state_bytes(sw.EULER_F64_FLAT, n) == 24 * n
    assert sw.sw_state_bytes(sw.EULER_F32_FLAT, n) == 24 * n
    for eq, per_cell in ((sw.HEAT_F64, 16), (sw.HEAT_F32, 12), (sw.EULER_F64, 56), (sw.EULER_F32, 44),
                         (sw.EULER_F64_FLAT, 48), (sw.EULER_F32_FLAT, 36)):
        assert sw.sw_workspace_bytes(eq, n, 0, sw.METHOD_SWEPT) == 2 * per_cell * n
    assert sw.sw_workspace_bytes(sw.EULER_F64_FLAT, n, 0, sw.METHOD_NAIVE) == 24 * n
    assert sw.sw_workspace_bytes(sw.HEAT_F64, n, 0, sw.METHOD_NAIVE) == 8 * n
    assert sw.sw_workspace_bytes(sw.EULER_F64, n, 0, sw.METHOD_NAIVE) == 32 * n
    assert sw.sw_workspace_bytes(sw.EULER_F64, n, 0, 9) == 0


def test_width_limits():
    for eq, per_cell, rad in ((sw.HEAT_F64, 16, 1), (sw.HEAT_F32, 12, 1), (sw.EULER_F64, 64, 1),
                              (sw.EULER_F32, 52, 1), (sw.EULER_F64_FLAT, 48, 2),
                              (sw.EULER_F32_FLAT, 36, 2)):
        wmax = sw.sw_max_width(eq)
        assert wmax % (2 * rad) == 0 and (wmax + 2 * rad) * per_cell <= 160 * 1024
        assert wmax <= 8192
    assert sw.sw_default_width(sw.HEAT_F64, 1 << 22) == 2048
    assert sw.sw_default_width(sw.EULER_F64, 1 << 22) == 1024
    assert sw.sw_default_width(sw.EULER_F32, 1 << 24) == 1024
    assert sw.sw_default_width(sw.HEAT_F32, 1 << 24) == 2048
    assert sw.sw_default_width(sw.HEAT_F64, 1000) == 500  # largest even divisor with n/W >= 2
    assert sw.sw_default_width(sw.HEAT_F64, 1001) == 0    # odd: no even divisor
    assert sw.sw_default_width(sw.HEAT_F64, 6) == 2
    # flattened Euler needs widths that are multiples of 4
    assert sw.sw_default_width(sw.EULER_F64_FLAT, 1 << 22) == 1024
    assert sw.sw_default_width(sw.EULER_F32_FLAT, 1 << 24) == 2048
    assert sw.sw_default_width(sw.EULER_F64_FLAT, 24) == 12
    assert sw.sw_default_width(sw.EULER_F64_FLAT, 18) == 0


def test_default_threads():
    # Euler tiles of 1000 cells and more: 512 threads; else whole waves up to 256
    for eq in (sw.EULER_F64, sw.EULER_F32, sw.EULER_F64_FLAT, sw.EULER_F32_FLAT):
        assert sw.sw_default_threads(eq, 1024) == 512
        assert sw.sw_default_threads(eq, 1000) == 512
        assert sw.sw_default_threads(eq, 992) == 256
        assert sw.sw_default_threads(eq, 2048) == 512
        assert sw.sw_default_threads(eq, 512) == 256
        assert sw.sw_default_threads(eq, 100) == 128
    assert sw.sw_default_threads(sw.KS_F64, 2048) == 512
    assert sw.sw_default_threads(sw.KS_F64, 1024) == 256
    assert sw.sw_default_threads(sw.HEAT_F64, 1024) == 256
    assert sw.sw_default_threads(sw.HEAT_F32, 2048) == 256
    assert sw.sw_default_threads(sw.HEAT_F64, 2) == 64
    assert sw.sw_default_threads(sw.EULER_F64_FLAT, 34) == 0   # not a multiple of 4
    assert sw.sw_default_threads(sw.HEAT_F64, 1 << 20) == 0    # wider than the LDS allows
    assert sw.sw_default_threads(9, 64) == 0


FAKE = 0x1000  # never dereferenced: every case below fails or returns before any HIP call


@pytest.mark.parametrize("fn", ["swept", "naive"])
@pytest.mark.parametrize("args,code", [
    ((9, 64, 1, 0.1, 1.0, FAKE), sw.SW_ERR_ARG),               # bad equation id
    ((sw.HEAT_F64, 2, 1, 0.1, 1.0, FAKE), sw.SW_ERR_ARG),      # too few cells
    ((sw.HEAT_F64, 64, -1, 0.1, 1.0, FAKE), sw.SW_ERR_ARG),    # negative steps
    ((sw.HEAT_F64, 64, 1, 0.0, 1.0, FAKE), sw.SW_ERR_ARG),     # dt <= 0
    ((sw.HEAT_F64, 64, 1, math.nan, 1.0, FAKE), sw.SW_ERR_ARG),
    ((sw.HEAT_F64, 64, 1, 0.1, math.inf, FAKE), sw.SW_ERR_ARG),
    ((sw.HEAT_F64, 64, 1, 0.1, -1.0, FAKE), sw.SW_ERR_ARG),
    ((sw.HEAT_F64, 64, 1, 0.1, 1.0, None), sw.SW_ERR_ARG),     # null state
    ((sw.HEAT_F64, 64, 1, 0.1, 1.0, FAKE + 8), sw.SW_ERR_ARG),  # misaligned
    ((sw.EULER_F32, 64, 0, 0.1, 1.0, FAKE), sw.SW_OK),        # zero steps: no-op
])
def test_host_validation(fn, args, code):
    f = sw.swept_solve if fn == "swept" else sw.naive_solve
    assert f(*args, None) == code
    if code != sw.SW_OK:
        assert sw.last_error()


@pytest.mark.parametrize("width", [3, 0 - 2, 6, 1024, 100000])
def test_invalid_width_rejected_on_host(width):
    # n = 1024: 6 does not divide it, 1024 leaves one tile, 100000 is too wide
    rc = sw.swept_solve_ex(sw.HEAT_F64, 1024, 5, 0.25, 1.0, FAKE, None, width=width)
    assert rc == sw.SW_ERR_ARG, sw.last_error()


def test_flat_width_must_be_multiple_of_four():
    rc = sw.swept_solve_ex(sw.EULER_F64_FLAT, 1024, 5, 0.1, 1.0, FAKE, None, width=34)
    assert rc == sw.SW_ERR_ARG
    assert sw.swept_solve(sw.EULER_F32_FLAT, 1026, 5, 0.1, 1.0, FAKE, None) == sw.SW_ERR_UNSUPPORTED


def test_no_valid_width_is_unsupported():
    assert sw.swept_solve(sw.HEAT_F64, 1001, 5, 0.25, 1.0, FAKE, None) == sw.SW_ERR_UNSUPPORTED
    # the classic method accepts any n >= 3
    assert sw.naive_solve(sw.HEAT_F64, 1001, 0, 0.25, 1.0, FAKE, None) == sw.SW_OK


def test_misaligned_workspace_rejected():
    rc = sw.swept_solve_ex(sw.HEAT_F64, 1024, 5, 0.25, 1.0, FAKE, None, width=64,
                           workspace=FAKE + 16, workspace_bytes=1 << 20)
    assert rc == sw.SW_ERR_ARG


def test_python_binding_names_match_c_abi():
    for name in ("swept_solve", "naive_solve", "swept_solve_ex", "naive_solve_ex",
                 "sw_state_bytes", "sw_workspace_bytes", "sw_max_width", "sw_default_width",
                 "sw_default_threads",
                 "sw_phase_count", "sw_phase_info", "sw_phase_interval", "sw_release"):
        assert callable(getattr(sw, name))
    assert ctypes.sizeof(sw.sw_opts) == 32


def test_launch_work_item_limit_rejected_on_host():
    # 2^31 cells in tiles of 64 with 256-thread workgroups: 2^33 work-items in one phase
    big = 1 << 31
    rc = sw.swept_solve_ex(sw.HEAT_F64, big, 5, 0.25, 1.0, FAKE, None, width=64, threads=256)
    assert rc == sw.SW_ERR_ARG and "work-items" in sw.last_error()
    # the classic kernels launch one work-item per cell
    assert sw.naive_solve(sw.HEAT_F64, 1 << 33, 5, 0.25, 1.0, FAKE, None) == sw.SW_ERR_ARG
    assert "2^32" in sw.last_error()
    assert sw.naive_solve(sw.EULER_F64, (1 << 32) - 255, 0, 0.1, 1.0, FAKE, None) == sw.SW_ERR_ARG
    # at the edge of the limit the call gets past the launch check (zero steps: no-op)
    assert sw.naive_solve(sw.EULER_F64, (1 << 32) - 256, 0, 0.1, 1.0, FAKE, None) == sw.SW_OK
    assert sw.swept_solve_ex(sw.HEAT_F64, big, 0, 0.25, 1.0, FAKE, None, width=2048,
                             threads=256) == sw.SW_OK


def test_workgroup_sizes_checked_on_host():
    for threads in (32, 96, 1024):
        rc = sw.swept_solve_ex(sw.EULER_F64, 4096, 5, 0.1, 1.0, FAKE, None, width=1024,
                               threads=threads)
        assert rc == sw.SW_ERR_ARG and "threads" in sw.last_error()
    for threads in (64, 128, 256, 512):  # accepted (zero steps: no device call)
        assert sw.swept_solve_ex(sw.EULER_F64, 4096, 0, 0.1, 1.0, FAKE, None, width=1024,
                                 threads=threads) == sw.SW_OK


def _ru(x, a=256):
    return (x + a - 1) // a * a


def test_batch_workspace_bytes_layout():
    """Header, problem table (96 bytes per entry), one 32-bit flag per tile,
    then both working-array copies of every problem, each part 256-aligned."""
    probs = [dict(eq=sw.HEAT_F64, width=64, n_cells=1024, n_steps=100, dt=0.25, dx=1.0,
                  d_state=FAKE),
             dict(eq=sw.EULER_F32, width=128, n_cells=3 * 1024, n_steps=7, dt=0.1, dx=1.0,
                  d_state=FAKE + 4096),
             dict(eq=sw.EULER_F64_FLAT, width=256, n_cells=1024, n_steps=1, dt=0.1, dx=1.0,
                  d_state=FAKE + 8192)]
    tiles = 1024 // 64 + 3 * 1024 // 128 + 1024 // 256
    arrays = 2 * _ru(1024 * 16) + 2 * _ru(3 * 1024 * 44) + 2 * _ru(1024 * 48)
    want = 256 + _ru(3 * 96) + _ru(4 * tiles) + arrays
    assert sw.sw_batch_workspace_bytes(probs) == want
    # the same list with one problem more changes every part
    more = probs + [dict(probs[0], d_state=FAKE + 12288)]
    assert sw.sw_batch_workspace_bytes(more) == (256 + _ru(4 * 96) + _ru(4 * (tiles + 16))
                                                 + arrays + 2 * _ru(1024 * 16))


def test_batch_workspace_checked_on_host():
    """swept_solve_batch rejects a missing, misaligned or short workspace and
    an invalid list before any HIP call (this runs without a GPU)."""
    probs = [dict(eq=sw.HEAT_F64, width=64, n_cells=1024, n_steps=100, dt=0.25, dx=1.0,
                  d_state=FAKE)]
    need = sw.sw_batch_workspace_bytes(probs)
    assert need > 0
    assert sw.swept_solve_batch(probs, None, need) == sw.SW_ERR_ARG
    assert "d_ws" in sw.last_error()
    assert sw.swept_solve_batch(probs, FAKE + 128, need) == sw.SW_ERR_ARG
    assert "aligned" in sw.last_error()
    assert sw.swept_solve_batch(probs, FAKE, need - 1) == sw.SW_ERR_ARG
    assert "smaller" in sw.last_error()
    assert sw.swept_solve_batch(probs, FAKE, need, threads=384) == sw.SW_ERR_ARG
    bad = [dict(probs[0], width=48)]  # does not divide 1024
    assert sw.sw_batch_workspace_bytes(bad) == 0
    assert sw.swept_solve_batch(bad, FAKE, need) == sw.SW_ERR_ARG
    # zero steps everywhere: nothing to launch, no device call
    idle = [dict(probs[0], n_steps=0)]
    assert sw.swept_solve_batch(idle, FAKE, sw.sw_batch_workspace_bytes(idle)) == sw.SW_OK


def test_batch_phase_count_bounded_on_host():
    """More than 2^31 - 2 swept phases cannot be numbered by the 32-bit tile
    flags: rejected on the host instead of truncated."""
    probs = [dict(eq=sw.HEAT_F64, width=4, n_cells=1024, n_steps=1 << 33, dt=0.25, dx=1.0,
                  d_state=FAKE)]
    assert sw.sw_batch_workspace_bytes(probs) == 0
    assert "phases" in sw.last_error()
    h = ctypes.c_void_p()
    arr = sw.problem_array(probs)
    assert sw.load().sw_batch_create(1, arr, None, ctypes.byref(h)) == sw.SW_ERR_ARG


def test_noalloc_limits_checked_on_host():
    """The allocation-free solve refuses, before any HIP call, a problem whose
    working arrays exceed its static arrays, and invalid arguments."""
    assert sw.NOALLOC_SCRATCH_BYTES == 64 * 1024 * 1024
    # heat binary64: 2 x 16 B per cell -> 2^21 cells fit, 2^21 + 2 do not
    rc = sw.swept_solve_noalloc(sw.HEAT_F64, (1 << 21) + 2, 5, 0.25, 1.0, FAKE, None)
    assert rc == sw.SW_ERR_ARG and "static" in sw.last_error()
    rc = sw.swept_solve_noalloc(sw.EULER_F64, 1 << 20, 5, 0.1, 1.0, FAKE, None)
    assert rc == sw.SW_ERR_ARG and "static" in sw.last_error()
    assert sw.swept_solve_noalloc(9, 1024, 5, 0.25, 1.0, FAKE, None) == sw.SW_ERR_ARG
    assert sw.swept_solve_noalloc(sw.HEAT_F64, 1024, -1, 0.25, 1.0, FAKE, None) == sw.SW_ERR_ARG
    assert sw.swept_solve_noalloc(sw.HEAT_F64, 1024, 5, 0.25, 1.0, None, None) == sw.SW_ERR_ARG


def test_work_factor_checked_on_host():
    """A shared solve is refused on the host when the work factor leaves the
    host no tile, for the classic method, and for negative values."""
    # 1024 cells in tiles of 64: 16 tiles; WF 1 with 8 threads: 16 // 9 = 1 tile each
    rc = sw.swept_solve_ex(sw.HEAT_F64, 1024, 5, 0.25, 1.0, FAKE, None, width=64, work_factor=9,
                           host_threads=8)
    assert rc == sw.SW_ERR_ARG and "no tile" in sw.last_error()
    rc = sw.swept_solve_ex(sw.HEAT_F64, 1024, 5, 0.25, 1.0, FAKE, None, width=64, work_factor=-1)
    assert rc == sw.SW_ERR_ARG
    rc = sw.swept_solve_ex(sw.HEAT_F64, 1024, 5, 0.25, 1.0, FAKE, None, width=64,
                           host_threads=100000)
    assert rc == sw.SW_ERR_ARG
    o = sw._opts(work_factor=2)
    rc = sw.load().naive_solve_ex(sw.HEAT_F64, 1024, 5, 0.25, 1.0, FAKE, None, ctypes.byref(o))
    assert rc == sw.SW_ERR_ARG and "swept" in sw.last_error()


def test_ks_sizes_widths_and_batch_refusal():
    n = 1 << 12
    assert sw.sw_state_bytes(sw.KS_F64, n) == 8 * n
    assert sw.sw_workspace_bytes(sw.KS_F64, n, 0, 0) == 2 * 16 * n  # two 16-byte slots
    assert sw.sw_default_width(sw.KS_F64, 1 << 24) == 2048
    assert sw.sw_default_width(sw.KS_F64, 24) == 12          # radius 2: multiples of 4
    assert sw.sw_default_width(sw.KS_F64, 18) == 0
    rc = sw.swept_solve_ex(sw.KS_F64, 1024, 5, 0.05, 1.0, FAKE, None, width=6)
    assert rc == sw.SW_ERR_ARG                                 # not a multiple of 4
    probs = (sw.sw_problem * 1)()
    probs[0] = sw.sw_problem(sw.KS_F64, 0, 4096, 10, 0.05, 1.0, FAKE)
    assert sw.load().sw_batch_workspace_bytes(1, probs) == 0
    assert "Kuramoto" in sw.last_error()
