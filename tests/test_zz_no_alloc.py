"""The allocation-free solve (swept_solve_noalloc, working arrays in the
library's static device array) against swept_solve with the library's own
working arrays, through the C ABI: two calls in a row, the second on a
smaller problem of another equation, each bit-identical to swept_solve and
to the oracle; a third call on a problem too large for the static arrays is
refused and leaves the state untouched."""
import numpy as np
import pytest

import oracle
import paper_1811_08282_amd as sw
from paper_1811_08282_amd.workloads import heat_ic, sod_tiled
from gpu_util import announce, pack

pytestmark = pytest.mark.gpu


def _pair(eq, host, steps, dt, dx):
    import torch
    a = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    b = a.clone()
    stream = torch.cuda.current_stream().cuda_stream
    n = host.shape[1]
    assert sw.swept_solve_noalloc(eq, n, steps, dt, dx, a.data_ptr(), stream) == sw.SW_OK, \
        sw.last_error()
    assert sw.swept_solve(eq, n, steps, dt, dx, b.data_ptr(), stream) == sw.SW_OK, sw.last_error()
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_solve_equals_swept_solve_twice_then_refuses_oversize():
    import torch
    # 1: heat binary64, 2^21 cells (the static arrays' limit), 3001 steps
    n = 1 << 21
    u0 = heat_ic(n, 11)
    announce("noalloc heat_f64", n, 3001)
    got, want = _pair(sw.HEAT_F64, pack(sw.HEAT_F64, u0), 3001, 0.25, 1.0)
    assert np.array_equal(got, want)
    span, steps = 16, 3001
    idx = np.arange(n // 2 - steps - 1, n // 2 + span + steps + 1) % n
    cone = oracle.heat_f64(u0[idx], steps, 0.25)[steps + 1: steps + 1 + span]
    assert np.array_equal(got[0][n // 2: n // 2 + span], cone)
    # 2: a smaller Euler binary64 problem right after (the arrays keep call 1's data)
    q0 = sod_tiled(1 << 14, 1 << 12)
    announce("noalloc euler_f64", q0.shape[1], 400)
    got, want = _pair(sw.EULER_F64, q0, 400, 0.1, 1.0)
    assert np.array_equal(got, want)
    assert np.array_equal(got, oracle.euler_f64(q0, 400, 0.1))
    # 3: binary32 heat with Kahan compensation, smaller again
    u1 = heat_ic(1 << 16, 12)
    announce("noalloc heat_f32", 1 << 16, 777)
    got, want = _pair(sw.HEAT_F32, pack(sw.HEAT_F32, u1), 777, 0.25, 1.0)
    assert np.array_equal(got, want)
    # 4: too large: refused before any device work, state unchanged
    big = torch.from_numpy(pack(sw.HEAT_F64, heat_ic((1 << 21) + 64, 13))).cuda()
    before = big.clone()
    rc = sw.swept_solve_noalloc(sw.HEAT_F64, (1 << 21) + 64, 10, 0.25, 1.0, big.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rc == sw.SW_ERR_ARG and "static" in sw.last_error()
    assert torch.equal(big, before)
