"""swept_solve runs heat grids of more than 1024 tiles of 1792 cells or more
as one persistent launch (the heat-only batch kernel, its phases overlapped)
when the caller gives no workspace, workgroup size or work factor; with a
workgroup size, fewer tiles or narrower ones it launches once per phase.  Both equal the classic solve bit for bit, in binary64 and
binary32.  A dependency wait of the persistent launch that runs out (forced
here from the host with a one-microsecond bound, SW_WAIT_LIMIT_US) leaves the
caller's state filled with NaN, and the next call runs normally.  The
autotuner weighs the persistent launch too (recorded as workgroup size 0),
and a record of either kind selects its route."""
import os

import numpy as np
import pytest

import paper_1811_08282_amd as sw
from paper_1811_08282_amd.workloads import heat_ic
from gpu_util import announce, pack

pytestmark = pytest.mark.gpu

N = 1 << 22  # 2048 tiles of 2048 cells


@pytest.mark.parametrize("eq", [sw.HEAT_F64, sw.HEAT_F32])
def test_persistent_and_phase_routes_equal_classic(eq):
    import torch
    steps = 2500
    host = pack(eq, heat_ic(N, 41))
    out = {}
    for name, kwargs in (("persistent", {}), ("phases", {"threads": 256}),
                         ("classic", {"method": "naive"})):
        announce("swept_solve route", eq, name, N, steps)
        t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
        sw.solve(eq, t, steps, 0.25, 1.0, **kwargs)
        torch.cuda.synchronize()
        out[name] = t.cpu().numpy()
    assert np.array_equal(out["persistent"], out["classic"])
    assert np.array_equal(out["phases"], out["classic"])


def test_aborted_persistent_launch_poisons_the_state():
    import torch
    host = pack(sw.HEAT_F64, heat_ic(1 << 22, 43))
    t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    announce("swept_solve forced abort")
    os.environ["SW_WAIT_LIMIT_US"] = "1"
    try:
        sw.solve(sw.HEAT_F64, t, 3000, 0.25, 1.0)
        torch.cuda.synchronize()
    finally:
        del os.environ["SW_WAIT_LIMIT_US"]
    assert torch.isnan(t).all().item()
    # the next call resets the launch's status and runs to the end
    t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    c = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    sw.solve(sw.HEAT_F64, t, 300, 0.25, 1.0)
    sw.solve(sw.HEAT_F64, c, 300, 0.25, 1.0, method="naive")
    torch.cuda.synchronize()
    assert torch.equal(t, c)


def test_autotune_weighs_the_persistent_launch():
    """On a heat grid of 2^22 cells the autotuner times the persistent launch
    beside the workgroup sizes at widths of 1792 and up (recorded as size 0);
    whichever wins, swept_solve with the record equals the classic solve."""
    import torch
    sw.sw_tune_clear()
    try:
        announce("autotune heat_f64 with the persistent launch", N)
        w, threads, ms = sw.sw_autotune(sw.HEAT_F64, N, 0)
        assert threads in (0, 64, 128, 256, 512) and N % w == 0 and ms > 0
        assert sw.sw_tuned_width(sw.HEAT_F64, N) == (w, threads)
        host = pack(sw.HEAT_F64, heat_ic(N, 45))
        t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
        c = torch.from_numpy(np.ascontiguousarray(host)).cuda()
        sw.solve(sw.HEAT_F64, t, 1500, 0.25, 1.0)
        sw.solve(sw.HEAT_F64, c, 1500, 0.25, 1.0, method="naive")
        torch.cuda.synchronize()
        assert torch.equal(t, c)
    finally:
        sw.sw_tune_clear()


_ROUTE_PROBE = """
import numpy as np, torch
import paper_1811_08282_amd as sw
from paper_1811_08282_amd.workloads import heat_ic
n = 1 << 22
print('tuned', sw.sw_tuned_width(sw.HEAT_F64, n), sw.sw_tuned_width(sw.EULER_F64, n),
      sw.sw_tuned_width(sw.HEAT_F64, 1 << 21), sw.sw_tuned_width(sw.HEAT_F64, 1 << 23), flush=True)
t = torch.from_numpy(heat_ic(n, 43).reshape(1, -1).copy()).cuda()
sw.solve(sw.HEAT_F64, t, 3000, 0.25, 1.0)
torch.cuda.synchronize()
print('nan', bool(torch.isnan(t).all().item()), bool(torch.isnan(t).any().item()), flush=True)
"""


@pytest.mark.parametrize("threads", [0, 256])
def test_tuned_record_selects_the_route(threads, tmp_path):
    """A record read from the tune cache file with workgroup size 0 sends
    swept_solve down the persistent launch (shown by the NaN a 1 us wait
    bound leaves), size 256 down the phase launches (no persistent launch,
    so nothing to abort).  Size 0 is refused for Euler, for heat grids of
    1024 tiles or fewer and for tiles narrower than 1792 cells."""
    import subprocess
    import sys
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = tmp_path / "tune.txt"
    path.write_text(f"{arch} {sw.HEAT_F64} {1 << 22} 2048 {threads} 1e-9\n"
                    f"{arch} {sw.EULER_F64} {1 << 22} 1024 0 1e-9\n"
                    f"{arch} {sw.HEAT_F64} {1 << 21} 2048 0 1e-9\n"
                    f"{arch} {sw.HEAT_F64} {1 << 23} 1024 0 1e-9\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, SWEPT_TUNE_CACHE=str(path), SW_WAIT_LIMIT_US="1", PYTHONPATH=root)
    announce("tuned route", threads)
    p = subprocess.run([sys.executable, "-c", _ROUTE_PROBE], env=env, capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 0, p.stderr
    lines = dict(line.split(" ", 1) for line in p.stdout.strip().splitlines())
    assert lines["tuned"] == f"(2048, {threads}) None None None"
    assert lines["nan"] == ("True True" if threads == 0 else "False False")
