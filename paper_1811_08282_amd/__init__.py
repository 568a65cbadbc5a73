"""Swept-rule stencil library for MI355X (gfx950) -- Python binding.

Thin ctypes marshalling over the C ABI in ``include/swept.h``; every step of
the computation runs in the HIP kernels of ``libswept.so``.  The functions
``swept_solve``, ``naive_solve`` (and the ``_ex`` forms) take raw device
pointers and a HIP stream handle exactly like the C functions; :func:`solve`
is a convenience wrapper for ``torch`` device tensors (torch provides device
memory and streams only).

The library must be built first (``python -m paper_1811_08282_amd.build``);
loading fails loudly when it is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswept.so")

# equation x precision x layout ids (sw_equation)
HEAT_F64, HEAT_F32, EULER_F64, EULER_F32, EULER_F64_FLAT, EULER_F32_FLAT, KS_F64 = range(7)
EQUATIONS = {"heat_f64": HEAT_F64, "heat_f32": HEAT_F32,
             "euler_f64": EULER_F64, "euler_f32": EULER_F32,
             "euler_f64_flat": EULER_F64_FLAT, "euler_f32_flat": EULER_F32_FLAT, "ks_f64": KS_F64}
# methods (sw_method)
METHOD_SWEPT, METHOD_NAIVE = 0, 1
# status codes (sw_status)
SW_OK, SW_ERR_ARG, SW_ERR_UNSUPPORTED, SW_ERR_HIP, SW_ERR_NOMEM, SW_ERR_CAPTURE = range(6)
STATUS_NAMES = {0: "SW_OK", 1: "SW_ERR_ARG", 2: "SW_ERR_UNSUPPORTED", 3: "SW_ERR_HIP",
                4: "SW_ERR_NOMEM", 5: "SW_ERR_CAPTURE"}


class SweptError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class sw_opts(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("threads", ctypes.c_int),
                ("d_workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("work_factor", ctypes.c_int), ("host_threads", ctypes.c_int)]


class sw_problem(ctypes.Structure):
    _fields_ = [("eq", ctypes.c_int), ("width", ctypes.c_int), ("n_cells", ctypes.c_int64),
                ("n_steps", ctypes.c_int64), ("dt", ctypes.c_double), ("dx", ctypes.c_double),
                ("d_state", ctypes.c_void_p)]


class sw_batch_opts(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int), ("threads", ctypes.c_int),
                ("wait_limit_us", ctypes.c_int64)]


_lib = None


def load() -> ctypes.CDLL:
    """Load ``libswept.so`` (raises if it has not been built).

    torch ships its own HIP runtime.  If the library were opened first, it
    would bind to the system HIP runtime and torch, imported later, would
    load its own: two runtimes on one GPU in one process, neither knowing the
    other's allocations.  So torch (when installed) is imported first; the
    library then binds to the runtime torch already loaded."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1811_08282_amd.build`")
    try:
        import torch  # noqa: F401  (loads torch's HIP runtime before the library)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    i64, i32, d, vp, sz = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
    solve_args = [i32, i64, i64, d, d, vp, vp]
    for name in ("swept_solve", "naive_solve", "swept_solve_noalloc"):
        getattr(lib, name).argtypes = solve_args
        getattr(lib, name).restype = i32
    for name in ("swept_solve_ex", "naive_solve_ex"):
        getattr(lib, name).argtypes = solve_args + [ctypes.POINTER(sw_opts)]
        getattr(lib, name).restype = i32
    lib.sw_state_bytes.argtypes = [i32, i64]
    lib.sw_state_bytes.restype = sz
    lib.sw_workspace_bytes.argtypes = [i32, i64, i32, i32]
    lib.sw_workspace_bytes.restype = sz
    lib.sw_max_width.argtypes = [i32]
    lib.sw_max_width.restype = i32
    lib.sw_default_width.argtypes = [i32, i64]
    lib.sw_default_width.restype = i32
    lib.sw_default_threads.argtypes = [i32, i32]
    lib.sw_default_threads.restype = i32
    lib.sw_phase_count.argtypes = [i64, i32, i32]
    lib.sw_phase_count.restype = i64
    lib.sw_phase_info.argtypes = [i64, i64, i32, i32, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                  ctypes.POINTER(i64)]
    lib.sw_phase_info.restype = i32
    lib.sw_phase_interval.argtypes = [i64, i64, i32, i32, i64, ctypes.POINTER(i32),
                                      ctypes.POINTER(i32)]
    lib.sw_phase_interval.restype = i32
    lib.sw_last_error.argtypes = []
    lib.sw_last_error.restype = ctypes.c_char_p
    lib.sw_release.argtypes = []
    lib.sw_release.restype = None
    lib.sw_autotune.argtypes = [i32, i64, i64, vp, ctypes.POINTER(sw_opts), ctypes.POINTER(d)]
    lib.sw_autotune.restype = i32
    lib.sw_tuned_width.argtypes = [i32, i64, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.sw_tuned_width.restype = i32
    lib.sw_tune_clear.argtypes = []
    lib.sw_tune_clear.restype = None
    lib.sw_batch_create.argtypes = [i32, ctypes.POINTER(sw_problem), ctypes.POINTER(sw_batch_opts),
                                    ctypes.POINTER(vp)]
    lib.sw_batch_create.restype = i32
    lib.sw_batch_run.argtypes = [vp, vp]
    lib.sw_batch_run.restype = i32
    lib.sw_batch_wait.argtypes = [vp, vp]
    lib.sw_batch_wait.restype = i32
    lib.sw_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(sz)]
    lib.sw_batch_info.restype = i32
    lib.sw_batch_width.argtypes = [vp, i32]
    lib.sw_batch_width.restype = i32
    lib.sw_batch_destroy.argtypes = [vp]
    lib.sw_batch_destroy.restype = None
    lib.swept_solve_batch.argtypes = [i32, ctypes.POINTER(sw_problem), vp, sz, vp]
    lib.swept_solve_batch.restype = i32
    lib.swept_solve_batch_ex.argtypes = [i32, ctypes.POINTER(sw_problem),
                                         ctypes.POINTER(sw_batch_opts), vp, sz, vp]
    lib.swept_solve_batch_ex.restype = i32
    lib.sw_batch_workspace_bytes.argtypes = [i32, ctypes.POINTER(sw_problem)]
    lib.sw_batch_workspace_bytes.restype = sz
    lib.sw_batch_check.argtypes = [vp, vp]
    lib.sw_batch_check.restype = i32
    lib.sw_batch_item_deps.argtypes = [i32, i32, i32, i32, ctypes.POINTER(i32)]
    lib.sw_batch_item_deps.restype = i32
    lib.sw_batch_autotune.argtypes = [i32, ctypes.POINTER(sw_problem), i64, vp,
                                      ctypes.POINTER(sw_batch_opts), ctypes.POINTER(d)]
    lib.sw_batch_autotune.restype = i32
    _lib = lib
    return lib


def last_error() -> str:
    return load().sw_last_error().decode()


def _opts(width: int = 0, workspace: int | None = None, workspace_bytes: int = 0,
          threads: int = 0, work_factor: int = 0, host_threads: int = 0):
    o = sw_opts()
    o.width = int(width)
    o.threads = int(threads)
    o.d_workspace = workspace
    o.workspace_bytes = int(workspace_bytes)
    o.work_factor = int(work_factor)
    o.host_threads = int(host_threads)
    return o


# ---- raw C-ABI mirrors (device pointers as ints) ---------------------------

def swept_solve(eq, n_cells, n_steps, dt, dx, d_state, stream=None) -> int:
    return load().swept_solve(eq, n_cells, n_steps, dt, dx, d_state, stream)


def naive_solve(eq, n_cells, n_steps, dt, dx, d_state, stream=None) -> int:
    return load().naive_solve(eq, n_cells, n_steps, dt, dx, d_state, stream)


# size of the static working arrays of swept_solve_noalloc (SW_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


def swept_solve_noalloc(eq, n_cells, n_steps, dt, dx, d_state, stream=None) -> int:
    return load().swept_solve_noalloc(eq, n_cells, n_steps, dt, dx, d_state, stream)


def swept_solve_ex(eq, n_cells, n_steps, dt, dx, d_state, stream=None, width=0,
                   workspace=None, workspace_bytes=0, threads=0, work_factor=0,
                   host_threads=0) -> int:
    o = _opts(width, workspace, workspace_bytes, threads, work_factor, host_threads)
    return load().swept_solve_ex(eq, n_cells, n_steps, dt, dx, d_state, stream, ctypes.byref(o))


def naive_solve_ex(eq, n_cells, n_steps, dt, dx, d_state, stream=None, workspace=None,
                   workspace_bytes=0) -> int:
    o = _opts(0, workspace, workspace_bytes)
    return load().naive_solve_ex(eq, n_cells, n_steps, dt, dx, d_state, stream, ctypes.byref(o))


def sw_state_bytes(eq, n_cells) -> int:
    return load().sw_state_bytes(eq, n_cells)


def sw_workspace_bytes(eq, n_cells, width=0, method=METHOD_SWEPT) -> int:
    return load().sw_workspace_bytes(eq, n_cells, width, method)


def sw_max_width(eq) -> int:
    return load().sw_max_width(eq)


def sw_default_width(eq, n_cells) -> int:
    return load().sw_default_width(eq, n_cells)


def sw_default_threads(eq, width) -> int:
    return load().sw_default_threads(eq, width)


def sw_phase_count(final_level, width, radius=1) -> int:
    return load().sw_phase_count(final_level, width, radius)


def sw_phase_info(k, final_level, width, radius=1):
    off, first, last = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = load().sw_phase_info(k, final_level, width, radius, ctypes.byref(off),
                              ctypes.byref(first), ctypes.byref(last))
    if rc:
        raise SweptError(rc, last_error())
    return off.value, first.value, last.value


def sw_phase_interval(k, final_level, width, level, radius=1):
    lo, hi = ctypes.c_int(), ctypes.c_int()
    rc = load().sw_phase_interval(k, final_level, width, radius, level, ctypes.byref(lo),
                                  ctypes.byref(hi))
    if rc:
        raise SweptError(rc, last_error())
    return lo.value, hi.value


def sw_release() -> None:
    load().sw_release()


# ---- autotuner -----------------------------------------------------------------

def sw_autotune(eq, n_cells, probe_steps=0, stream=None):
    """Returns (width, threads, ms_per_cell_update); threads 0 names the
    persistent launch (heat grids of more than 1024 tiles of 1792 cells or
    more).  Raises on failure."""
    best = sw_opts()
    ms = ctypes.c_double()
    rc = load().sw_autotune(eq, n_cells, probe_steps, stream, ctypes.byref(best), ctypes.byref(ms))
    if rc:
        raise SweptError(rc, last_error())
    return best.width, best.threads, ms.value


def sw_tuned_width(eq, n_cells):
    """(width, threads) recorded for (current device, eq, n_cells), or None
    (threads 0: the persistent launch)."""
    w, t = ctypes.c_int(), ctypes.c_int()
    rc = load().sw_tuned_width(eq, n_cells, ctypes.byref(w), ctypes.byref(t))
    return (w.value, t.value) if rc == SW_OK else None


def sw_tune_clear() -> None:
    load().sw_tune_clear()


# ---- batched persistent launch ----------------------------------------------------

def problem_array(problems):
    """List of dicts/tuples -> ctypes array of sw_problem."""
    arr = (sw_problem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = sw_problem(*p) if isinstance(p, (tuple, list)) else sw_problem(**p)
    return arr


def sw_batch_item_deps(phase, tile, tiles, single_phase=0):
    deps = (ctypes.c_int * 3)()
    n = load().sw_batch_item_deps(phase, tile, tiles, single_phase, deps)
    if n < 0:
        raise SweptError(SW_ERR_ARG, "invalid item")
    return list(deps[:n])


class Batch:
    """Owner of an sw_batch handle (see include/swept.h)."""

    def __init__(self, problems, blocks_per_cu=0, wait_limit_us=0, threads=0):
        self._arr = problem_array(problems)
        opts = sw_batch_opts(int(blocks_per_cu), int(threads), int(wait_limit_us))
        h = ctypes.c_void_p()
        rc = load().sw_batch_create(len(self._arr), self._arr, ctypes.byref(opts), ctypes.byref(h))
        if rc:
            raise SweptError(rc, last_error())
        self.handle = h

    def run(self, stream=None) -> None:
        rc = load().sw_batch_run(self.handle, stream)
        if rc:
            raise SweptError(rc, last_error())

    def wait(self, stream=None) -> int:
        return load().sw_batch_wait(self.handle, stream)

    def info(self):
        items, blocks, nbytes = ctypes.c_int64(), ctypes.c_int(), ctypes.c_size_t()
        load().sw_batch_info(self.handle, ctypes.byref(items), ctypes.byref(blocks),
                             ctypes.byref(nbytes))
        return items.value, blocks.value, nbytes.value

    def width(self, i) -> int:
        return load().sw_batch_width(self.handle, i)

    def close(self) -> None:
        if self.handle:
            load().sw_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sw_batch_autotune(problems, probe_steps=0, stream=None, threads=0):
    """Tune the batched launch (see include/swept.h): the problems' states are
    only read; every problem given with width 0 gets the chosen width written
    back into its dict.  ``threads`` = 0 tries 256- and 512-thread workgroups,
    else only that size.  Returns (blocks_per_cu, threads, ms per cell-update
    of the fastest probe); raises on failure."""
    arr = problem_array(problems)
    best = sw_batch_opts()
    best.threads = int(threads)
    ms = ctypes.c_double()
    rc = load().sw_batch_autotune(len(arr), arr, int(probe_steps), stream, ctypes.byref(best),
                                  ctypes.byref(ms))
    if rc:
        raise SweptError(rc, last_error())
    for p, a in zip(problems, arr):
        if isinstance(p, dict) and not p.get("width"):
            p["width"] = a.width
    return best.blocks_per_cu, best.threads, ms.value


def sw_batch_workspace_bytes(problems) -> int:
    """Device workspace bytes swept_solve_batch needs for ``problems`` (0 if invalid)."""
    arr = problem_array(problems)
    return load().sw_batch_workspace_bytes(len(arr), arr)


def swept_solve_batch(problems, d_ws, ws_bytes, stream=None, blocks_per_cu=0, threads=0,
                      wait_limit_us=0) -> int:
    """One persistent launch of ``problems`` in the caller's workspace ``d_ws``
    (a device pointer of at least ``sw_batch_workspace_bytes(problems)``
    bytes); asynchronous, allocates nothing.  Returns the status code."""
    arr = problem_array(problems)
    if blocks_per_cu or threads or wait_limit_us:
        opts = sw_batch_opts(int(blocks_per_cu), int(threads), int(wait_limit_us))
        return load().swept_solve_batch_ex(len(arr), arr, ctypes.byref(opts), d_ws, int(ws_bytes),
                                           stream)
    return load().swept_solve_batch(len(arr), arr, d_ws, int(ws_bytes), stream)


def sw_batch_check(d_ws, stream=None) -> int:
    """Wait for ``stream``; SW_ERR_HIP if the last launch in ``d_ws`` aborted."""
    return load().sw_batch_check(d_ws, stream)


# ---- torch convenience -----------------------------------------------------

def substeps(eq: int) -> int:
    return {EULER_F64: 4, EULER_F32: 4, EULER_F64_FLAT: 2, EULER_F32_FLAT: 2}.get(eq, 1)


def radius(eq: int) -> int:
    """Stencil radius of one sub-step (2 for the flattened Euler layout and
    Kuramoto-Sivashinsky)."""
    return 2 if eq in (EULER_F64_FLAT, EULER_F32_FLAT, KS_F64) else 1


def is_f64(eq: int) -> bool:
    return eq in (HEAT_F64, EULER_F64, EULER_F64_FLAT, KS_F64)


def state_dtype(eq: int):
    import torch
    return torch.float64 if is_f64(eq) else torch.float32


def state_rows(eq: int) -> int:
    """Arrays of n_cells in the state buffer (see include/swept.h)."""
    return {HEAT_F64: 1, HEAT_F32: 2, EULER_F64: 3, EULER_F32: 6,
            EULER_F64_FLAT: 3, EULER_F32_FLAT: 6, KS_F64: 1}[eq]


def solve(eq: int, state, n_steps: int, dt: float, dx: float, method: str = "swept",
          width: int = 0, workspace=None, stream=None, threads: int = 0, work_factor: int = 0,
          host_threads: int = 0) -> None:
    """Advance a torch device tensor of shape (rows, n_cells) in place.

    ``rows`` is :func:`state_rows`; the dtype is float64 for *_F64 and float32
    for *_F32.  Runs on ``stream`` (default: torch's current stream).
    ``work_factor`` > 0 shares the swept solve with ``host_threads`` host
    threads (sw_opts.work_factor); the call then returns when it is done.
    """
    import torch
    if not state.is_cuda or not state.is_contiguous():
        raise ValueError("state must be a contiguous device tensor")
    if state.dtype != state_dtype(eq) or state.dim() != 2 or state.shape[0] != state_rows(eq):
        raise ValueError(f"state must have shape ({state_rows(eq)}, n) and dtype {state_dtype(eq)}")
    n = state.shape[1]
    s = stream if stream is not None else torch.cuda.current_stream()
    handle = s.cuda_stream
    ws_ptr = workspace.data_ptr() if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    if method == "swept":
        rc = swept_solve_ex(eq, n, n_steps, dt, dx, state.data_ptr(), handle, width, ws_ptr,
                            ws_bytes, threads, work_factor, host_threads)
    elif method == "naive":
        rc = naive_solve_ex(eq, n, n_steps, dt, dx, state.data_ptr(), handle, ws_ptr, ws_bytes)
    else:
        raise ValueError("method must be 'swept' or 'naive'")
    if rc != SW_OK:
        raise SweptError(rc, last_error())
