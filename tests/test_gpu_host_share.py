"""The swept solve shared between the GPU and host threads (the GPU work
factor of Sec. 4.2, Eq. 1): a contiguous range of tiles runs on host threads
with host-compiled copies of the cell arithmetic and the seams cross through
pinned host memory once per phase.  Every equation id, several work factors
and thread counts, step counts ending in cut phases: the result equals
swept_solve and the oracle bit for bit."""
import numpy as np
import pytest

import oracle
import paper_1811_08282_amd as sw
from paper_1811_08282_amd.workloads import heat_ic, sod_tiled
from gpu_util import announce, pack

pytestmark = pytest.mark.gpu


def _oracle(eq, host, steps, dt):
    if eq == sw.HEAT_F64:
        return oracle.heat_f64(host[0], steps, dt).reshape(1, -1)
    if eq == sw.KS_F64:
        return oracle.ks_f64(host[0], steps, dt, 1.0).reshape(1, -1)
    if eq == sw.HEAT_F32:
        return np.stack(oracle.heat_f32(host[0], host[1], steps, dt))
    if eq in (sw.EULER_F64, sw.EULER_F64_FLAT):
        return oracle.euler_f64(host, steps, dt)
    q, c = oracle.euler_f32(host[:3], host[3:], steps, dt)
    return np.concatenate([q, c])


CASES = [
    # eq, n, width, steps, work factor, host threads
    (sw.HEAT_F64, 4096, 256, 777, 1, 3), (sw.HEAT_F64, 4096, 256, 777, 4, 1),
    (sw.HEAT_F64, 4096, 256, 129, 2, 2), (sw.HEAT_F64, 4096, 256, 1, 2, 2),
    (sw.HEAT_F32, 4096, 256, 777, 1, 3), (sw.HEAT_F32, 6144, 512, 1000, 3, 2),
    (sw.EULER_F64, 8192, 512, 300, 1, 3), (sw.EULER_F64, 8192, 512, 77, 5, 2),
    (sw.EULER_F32, 8192, 512, 300, 2, 2),
    (sw.EULER_F64_FLAT, 8192, 512, 300, 1, 3), (sw.EULER_F32_FLAT, 8192, 512, 300, 2, 2),
    (sw.KS_F64, 8192, 512, 500, 1, 3), (sw.KS_F64, 8192, 512, 129, 4, 2),
]


@pytest.mark.parametrize("eq,n,width,steps,wf,threads", CASES)
def test_shared_solve_equals_swept_solve_and_oracle(eq, n, width, steps, wf, threads):
    import torch
    if eq in (sw.HEAT_F64, sw.HEAT_F32):
        q0, dt = heat_ic(n, n + steps), 0.25
    elif eq == sw.KS_F64:
        q0, dt = 0.1 * heat_ic(n, n + steps), 0.02
    else:
        q0, dt = sod_tiled(n, 2048), 0.1
    host = pack(sw.EULER_F32 if eq == sw.EULER_F32_FLAT else
                (sw.EULER_F64 if eq == sw.EULER_F64_FLAT else
                 (sw.HEAT_F64 if eq == sw.KS_F64 else eq)), q0)
    announce("host share", eq, n, width, steps, "WF", wf, "threads", threads)
    a = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    b = a.clone()
    sw.solve(eq, a, steps, dt, 1.0, method="swept", width=width, work_factor=wf,
             host_threads=threads)
    sw.solve(eq, b, steps, dt, 1.0, method="swept", width=width)
    torch.cuda.synchronize()
    got, alone = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(got, alone)
    assert np.array_equal(got, _oracle(eq, host, steps, dt))


def test_shared_solve_in_chunks_and_on_another_stream():
    """Two shared calls of n1 and n2 steps equal one swept solve of n1 + n2,
    also on a stream other than the default one."""
    import torch
    n, w = 8192, 512
    host = pack(sw.HEAT_F64, heat_ic(n, 99))
    a = torch.from_numpy(host.copy()).cuda()
    b = a.clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        sw.solve(sw.HEAT_F64, a, 300, 0.25, 1.0, width=w, work_factor=3, host_threads=2)
        sw.solve(sw.HEAT_F64, a, 451, 0.25, 1.0, width=w, work_factor=3, host_threads=2)
    s.synchronize()
    sw.solve(sw.HEAT_F64, b, 751, 0.25, 1.0, width=w)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
