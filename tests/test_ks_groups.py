"""CPU replay of the Kuramoto-Sivashinsky level sweep's grouping: each thread
updates four consecutive cells, loading their eight-cell neighbourhood as
four 16-byte LDS loads and storing the four results as two 16-byte stores.
For every width the library accepts for the equation (multiples of 4) and
every level of the first and of a diamond phase, the groups must tile the
level's window exactly, start on an even LDS cell (so both 16-byte accesses
are aligned, the second slot starting W + 4 cells after the first), and
read only cells of the slot.  A plain replay of the same groups with the
scheme's per-cell formula must equal the per-cell sweep bit for bit."""
import numpy as np
import pytest

import paper_1811_08282_amd as sw

R = 2
CELLS = 4


def _windows(w, first_phase):
    """(lo, hi) LDS windows of every level of one phase, in order."""
    h = w // (2 * R)
    j_first = 1 if first_phase else 2 - h
    for j in range(j_first, h + 1):
        m = R * abs(j - 1)
        yield m + R, w - m + R


def _second(l, m, r):
    return (r - m) + (l - m)


def _flux(u):
    return 0.5 * (u * u)


def _update(u, a, b, c):
    """ks_update of the five values u[0..4] (the scheme as the kernel writes it)."""
    sm, s0, sp = _second(u[0], u[1], u[2]), _second(u[1], u[2], u[3]), _second(u[2], u[3], u[4])
    q = (sp - s0) + (sm - s0)
    return u[2] - ((a * (_flux(u[3]) - _flux(u[1])) + b * s0) + c * q)


def _group(u8, a, b, c):
    """The four-cell group: shared second differences and fluxes."""
    sd = [_second(u8[k], u8[k + 1], u8[k + 2]) for k in range(CELLS + 2)]
    fl = [_flux(u8[k + 1]) for k in range(CELLS + 2)]
    out = []
    for k in range(CELLS):
        q = (sd[k + 2] - sd[k + 1]) + (sd[k] - sd[k + 1])
        out.append(u8[k + 2] - ((a * (fl[k + 2] - fl[k]) + b * sd[k + 1]) + c * q))
    return out


def test_widths_are_multiples_of_four_and_slots_stay_aligned():
    wmax = sw.sw_max_width(sw.KS_F64)
    assert wmax % 4 == 0
    # n = 2W: W itself is the width the library picks for n exactly when it
    # accepts W (up to its preferred 2048; no wider width divides n twice)
    for w in range(4, 2049, 2):
        ok = sw.sw_default_width(sw.KS_F64, 2 * w) == w
        assert ok == (w % 4 == 0), w
    # the second slot starts W + 4 doubles after the first: a 32-byte multiple
    assert all((w + 2 * R) * 8 % 32 == 0 for w in range(4, wmax + 1, 4))


@pytest.mark.parametrize("first_phase", [True, False])
def test_groups_tile_every_window_aligned_and_in_bounds(first_phase):
    for w in list(range(4, 260, 4)) + [1020, 2044, 2048, 4096, sw.sw_max_width(sw.KS_F64)]:
        wp = w + 2 * R
        for lo, hi in _windows(w, first_phase):
            assert (hi - lo) % CELLS == 0 and lo % 2 == 0, (w, lo, hi)
            for x0 in range(lo, hi, CELLS):
                assert (x0 - 2) % 2 == 0 and x0 % 2 == 0
                assert 0 <= x0 - 2 and x0 + CELLS + 2 <= wp, (w, x0)


@pytest.mark.parametrize("w", [4, 8, 12, 36, 100])
def test_grouped_sweep_equals_per_cell_sweep(w):
    rng = np.random.default_rng(w)
    a, b, c = 0.01, 0.02, 0.02
    for first_phase in (True, False):
        s = [rng.uniform(-1, 1, w + 2 * R), rng.uniform(-1, 1, w + 2 * R)]
        t = [s[0].copy(), s[1].copy()]
        for lv, (lo, hi) in enumerate(_windows(w, first_phase)):
            src, dst = lv & 1, (lv + 1) & 1
            for i in range(lo, hi):
                s[dst][i] = _update(s[src][i - 2:i + 3], a, b, c)
            for x0 in range(lo, hi, CELLS):
                t[dst][x0:x0 + CELLS] = _group(t[src][x0 - 2:x0 + CELLS + 2], a, b, c)
            assert np.array_equal(s[dst], t[dst]), (w, first_phase, lv)
