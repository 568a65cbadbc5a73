"""GPU tests of the library's stream handling: every (device, stream) pair
keeps its own cached working arrays, so solves enqueued on two streams at
once stay independent; a cache that grows on a stream with work in flight,
and sw_release between calls, leave results unchanged.  Every result is
compared with the oracle bit for bit."""
import numpy as np
import pytest

import oracle
import paper_1811_08282_amd as sw
from paper_1811_08282_amd.workloads import heat_ic, sod_tiled
from gpu_util import announce, pack

pytestmark = pytest.mark.gpu


def _device(torch, host):
    t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    torch.cuda.current_stream().synchronize()  # the copy is done before other streams use t
    return t


def test_two_streams_in_flight_use_their_own_working_arrays():
    import torch
    u0 = heat_ic(8192, 41)
    q0 = sod_tiled(4096, 1024)
    q0[1] += 0.05 * q0[0]
    heat = _device(torch, pack(sw.HEAT_F64, u0))
    euler = _device(torch, pack(sw.EULER_F64, q0))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    announce("two streams: heat_f64 8192 on one, euler_f64 4096 on the other")
    # interleaved enqueues, no synchronisation until the end
    for _ in range(3):
        sw.solve(sw.HEAT_F64, heat, 70, 0.25, 1.0, width=512, stream=s1)
        sw.solve(sw.EULER_F64, euler, 40, 0.1, 1.0, width=256, stream=s2)
    s1.synchronize()
    s2.synchronize()
    assert np.array_equal(heat.cpu().numpy()[0], oracle.heat_f64(u0, 210, 0.25))
    assert np.array_equal(euler.cpu().numpy(), oracle.euler_f64(q0, 120, 0.1))


def test_growing_cache_with_work_in_flight_and_release():
    import torch
    small = heat_ic(1024, 42)
    large = heat_ic(1 << 16, 43)
    q0 = sod_tiled(8192, 2048)
    a = _device(torch, pack(sw.HEAT_F64, small))
    b = _device(torch, pack(sw.HEAT_F64, large))
    c = _device(torch, pack(sw.EULER_F64, q0))
    announce("cache growth on one stream: heat 1024, heat 65536, euler 8192")
    sw.sw_release()
    sw.solve(sw.HEAT_F64, a, 300, 0.25, 1.0)   # small arrays cached
    sw.solve(sw.HEAT_F64, b, 300, 0.25, 1.0)   # grows while the first solve may still run
    sw.solve(sw.EULER_F64, c, 50, 0.1, 1.0)    # grows again (56-byte structs)
    sw.solve(sw.HEAT_F64, a, 300, 0.25, 1.0)   # the grown arrays serve the small grid too
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy()[0], oracle.heat_f64(small, 600, 0.25))
    assert np.array_equal(b.cpu().numpy()[0], oracle.heat_f64(large, 300, 0.25))
    assert np.array_equal(c.cpu().numpy(), oracle.euler_f64(q0, 50, 0.1))
    announce("after sw_release")
    sw.sw_release()
    sw.solve(sw.EULER_F64, c, 50, 0.1, 1.0)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), oracle.euler_f64(q0, 100, 0.1))
