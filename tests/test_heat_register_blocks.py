"""CPU replay of the heat kernels' register-blocked level sweep against the
plain level sweep, bit for bit, on the two level slots of every tile cell:
up triangles, diamonds and flat cuts, odd and even W/2 (both level parities
at the block starts), windows narrow enough to fall back to the plain sweep,
and workgroups of one to eight waves (wide windows needing more rows than
the waves hold fall back too)."""
import numpy as np
import pytest

from heat_rb_emulator import blocked_levels, plain_levels


def _phase(w, k, final_level, seed, waves):
    h = w // 2
    base = (k - 1) * h
    j_first = 1 if k == 1 else 2 - h
    j_last = min(h, final_level - base)
    rng = np.random.default_rng(seed)
    slots = rng.uniform(-1, 1, size=(2, w + 2))
    a = {0: slots[0].copy(), 1: slots[1].copy()}
    b = {0: slots[0].copy(), 1: slots[1].copy()}
    plain_levels(a, w, base, range(j_first, j_last + 1), 0.25)
    blocked_levels(b, w, base, j_first, j_last, 0.25, waves=waves)
    for p in (0, 1):
        assert np.array_equal(a[p][1:w + 1], b[p][1:w + 1]), (w, k, final_level, waves, p)


@pytest.mark.parametrize("w", [20, 22, 64, 66, 130, 518, 1030])
def test_blocked_sweep_equals_level_sweep(w):
    h = w // 2
    for k in (1, 2, 3):
        for final in (10 ** 9, (k - 1) * h + 1, (k - 1) * h + 2, (k - 1) * h + h - 1,
                      (k - 1) * h + 7):
            if final > (k - 2) * h:
                _phase(w, k, final, seed=w * 31 + k * 7 + final % 1009, waves=4)


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_blocked_sweep_every_workgroup_size(waves):
    for w in (518, 2048):
        _phase(w, 2, 10 ** 9, seed=waves + w, waves=waves)
