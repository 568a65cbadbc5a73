"""Host emulation of the swept schedule the kernels run (no GPU).

The phase geometry comes from the library itself (sw_phase_count /
sw_phase_info / sw_phase_interval, which evaluate the same inline functions
the phase kernels use).  The emulator replays it exactly as a kernel does --
each tile snapshots its W cells plus one halo per side from the previous
phase's array, sweeps its window of levels, and writes its W cells to the
next array -- with an opaque hash as the cell update, and checks that:

* every (cell, level) is computed exactly once and from neighbours that hold
  the needed level (the two-slot struct of the heat kernels, the
  Q0 / Q1 / Pr struct of the Euler kernels);
* the result equals plain step-by-step evaluation of the same update.

A wrong window, offset, halo or slot choice changes the hash.
"""
import random

import pytest

import paper_1811_08282_amd as sw

MASK = (1 << 61) - 1


def _h(*xs):
    v = 0x9E3779B97F4A7C15
    for x in xs:
        v = ((v ^ (x & MASK)) * 0x100000001B3 + 0x632BE59BD9B4E019) & MASK
        v ^= v >> 29
    return v


def _phases(final_level, width, radius=1):
    k_count = sw.sw_phase_count(final_level, width, radius)
    for k in range(1, k_count + 1):
        off, first, last = sw.sw_phase_info(k, final_level, width, radius)
        yield k, k_count, off, first, last


# ---- heat-like: one value per level, two slots by level parity --------------

def _naive_heat(u0, levels):
    n = len(u0)
    u = list(u0)
    for m in range(1, levels + 1):
        u = [_h(u[i - 1], u[i], u[(i + 1) % n], m) for i in range(n)]
    return u


def _swept_heat(u0, levels, width):
    n = len(u0)
    # arrays hold (slot0, slot1, top level) per cell
    cur = [(v, None, 0) for v in u0]
    computed = set()
    for k, k_count, off, first, last in _phases(levels, width):
        nxt = [None] * n
        for t0 in range(off, off + n, width):
            idx = [(t0 - 1 + i) % n for i in range(width + 2)]
            s = [[cur[g][0], cur[g][1]] for g in idx]
            top = [cur[g][2] for g in idx]
            for m in range(first, last + 1):
                lo, hi = sw.sw_phase_interval(k, levels, width, m)
                assert hi - lo == width - 2 * abs(m - (k - 1) * (width // 2) - 1)
                new = {}
                for o in range(lo, hi):
                    i = o + 1
                    assert top[i] == m - 1, "cell not at the previous level"
                    for nb in (i - 1, i + 1):
                        assert top[nb] in (m - 1, m), "neighbour level not in the struct"
                    src = (m - 1) & 1
                    new[i] = _h(s[i - 1][src], s[i][src], s[i + 1][src], m)
                    key = (idx[i], m)
                    assert key not in computed, "cell-level computed twice"
                    computed.add(key)
                for i, v in new.items():
                    s[i][m & 1] = v
                    top[i] = m
            for i in range(1, width + 1):
                nxt[idx[i]] = (s[i][0], s[i][1], top[i])
        assert all(c is not None for c in nxt)
        cur = nxt
    assert all(c[2] == levels for c in cur)
    assert len(computed) == n * levels
    return [c[levels & 1] for c in cur]


@pytest.mark.parametrize("n,width", [(8, 2), (8, 4), (12, 6), (16, 8), (64, 8), (64, 32),
                                     (96, 16), (128, 64), (36, 18)])
def test_heat_schedule_equals_stepping(n, width):
    rng = random.Random(n * 1000 + width)
    u0 = [rng.getrandbits(60) for _ in range(n)]
    h = width // 2
    for levels in sorted({0, 1, 2, h - 1, h, h + 1, 2 * h, 3 * h + 1, 5 * h - 1,
                          rng.randint(1, 6 * h)}):
        if levels < 0:
            continue
        assert _swept_heat(u0, levels, width) == _naive_heat(u0, levels)


# ---- Euler-like: one struct (Q0, Q1, Pr) per cell, four sub-step types -----------

def _euler_update(t, m, c, left, right):
    """c, left, right: dicts with Q0, Q1, Pr; returns (field, value) written."""
    if t == 0:
        return "Pr", _h(left["Q0"], c["Q0"], right["Q0"], m)
    if t == 1:
        return "Q1", _h(left["Q0"], c["Q0"], right["Q0"], left["Pr"], c["Pr"], right["Pr"], m)
    if t == 2:
        return "Pr", _h(left["Q1"], c["Q1"], right["Q1"], m)
    return "Q0", _h(c["Q0"], left["Q1"], c["Q1"], right["Q1"], left["Pr"], c["Pr"], right["Pr"], m)


def _naive_euler(q0, levels):
    n = len(q0)
    st = [{"Q0": v, "Q1": 0, "Pr": 0} for v in q0]
    for m in range(1, levels + 1):
        t = (m - 1) & 3
        upd = [_euler_update(t, m, st[i], st[i - 1], st[(i + 1) % n]) for i in range(n)]
        for i, (f, v) in enumerate(upd):
            st[i][f] = v
    return [c["Q0"] for c in st]


def _swept_euler(q0, levels, width):
    n = len(q0)
    cur = [({"Q0": v, "Q1": 0, "Pr": 0}, 0) for v in q0]
    for k, k_count, off, first, last in _phases(levels, width):
        nxt = [None] * n
        for t0 in range(off, off + n, width):
            idx = [(t0 - 1 + i) % n for i in range(width + 2)]
            st = [dict(cur[g][0]) for g in idx]
            top = [cur[g][1] for g in idx]
            for m in range(first, last + 1):
                lo, hi = sw.sw_phase_interval(k, levels, width, m)
                t = (m - 1) & 3
                upd = {}
                for o in range(lo, hi):
                    i = o + 1
                    assert top[i] == m - 1 and top[i - 1] in (m - 1, m) and top[i + 1] in (m - 1, m)
                    upd[i] = _euler_update(t, m, st[i], st[i - 1], st[i + 1])
                for i, (f, v) in upd.items():
                    st[i][f] = v
                    top[i] = m
            for i in range(1, width + 1):
                nxt[idx[i]] = (st[i], top[i])
        cur = nxt
    assert all(c[1] == levels for c in cur)
    return [c[0]["Q0"] for c in cur]


@pytest.mark.parametrize("n,width", [(8, 2), (16, 4), (24, 8), (64, 16), (64, 32), (40, 10)])
def test_euler_struct_schedule_equals_stepping(n, width):
    rng = random.Random(7 * n + width)
    q0 = [rng.getrandbits(60) for _ in range(n)]
    h = width // 2
    for steps in sorted({0, 1, 2, 3, rng.randint(1, 3 * h)}):
        levels = 4 * steps
        assert _swept_euler(q0, levels, width) == _naive_euler(q0, levels)


def test_phase_counts_match_the_paper_structure():
    # F a multiple of H: Up Triangle, F/H - 1 Diamonds, Down Triangle
    assert sw.sw_phase_count(1000 * 32, 64) == 1000 + 1
    assert sw.sw_phase_count(0, 64) == 0
    assert sw.sw_phase_count(1, 64) == 1
    assert sw.sw_phase_count(33, 64) == 2
    assert sw.sw_phase_count(34, 64) == 3
    assert sw.sw_phase_count(5, 3) == -1
    # a full diamond computes W^2/2 cell-levels
    w, levels = 64, 10 * 32
    total = 0
    off, first, last = sw.sw_phase_info(3, levels, w)
    for m in range(first, last + 1):
        lo, hi = sw.sw_phase_interval(3, levels, w, m)
        total += hi - lo
    assert off == 0 and total == w * w // 2


# ---- radius 2 (the flattened Euler layout): five-point sub-steps ---------------

def _naive_r2(u0, levels):
    n = len(u0)
    u = list(u0)
    for m in range(1, levels + 1):
        u = [_h(u[i - 2], u[i - 1], u[i], u[(i + 1) % n], u[(i + 2) % n], m) for i in range(n)]
    return u


def _swept_r2(u0, levels, width):
    """Two-slot struct, halos of two cells, margins doubled."""
    n, R = len(u0), 2
    cur = [(v, None, 0) for v in u0]
    computed = set()
    for k, k_count, off, first, last in _phases(levels, width, R):
        nxt = [None] * n
        for t0 in range(off, off + n, width):
            idx = [(t0 - R + i) % n for i in range(width + 2 * R)]
            s = [[cur[g][0], cur[g][1]] for g in idx]
            top = [cur[g][2] for g in idx]
            for m in range(first, last + 1):
                lo, hi = sw.sw_phase_interval(k, levels, width, m, R)
                j = m - (k - 1) * (width // (2 * R))
                assert (lo, hi) == (R * abs(j - 1), width - R * abs(j - 1))
                new = {}
                for o in range(lo, hi):
                    i = o + R
                    assert top[i] == m - 1
                    for nb in (i - 2, i - 1, i + 1, i + 2):
                        assert top[nb] in (m - 1, m), "neighbour level not in the struct"
                    src = (m - 1) & 1
                    new[i] = _h(*(s[i + d][src] for d in (-2, -1, 0, 1, 2)), m)
                    assert (idx[i], m) not in computed
                    computed.add((idx[i], m))
                for i, v in new.items():
                    s[i][m & 1] = v
                    top[i] = m
            for i in range(R, width + R):
                nxt[idx[i]] = (s[i][0], s[i][1], top[i])
        cur = nxt
    assert all(c[2] == levels for c in cur) and len(computed) == n * levels
    return [c[levels & 1] for c in cur]


@pytest.mark.parametrize("n,width", [(8, 4), (16, 4), (16, 8), (24, 12), (64, 16), (96, 32)])
def test_radius2_schedule_equals_stepping(n, width):
    rng = random.Random(n * 77 + width)
    u0 = [rng.getrandbits(60) for _ in range(n)]
    h = width // 4
    for levels in sorted({0, 1, 2, h, h + 1, 3 * h + 1, rng.randint(1, 6 * h)}):
        assert _swept_r2(u0, levels, width) == _naive_r2(u0, levels)


def _flat_update(t, m, c, nb):
    """Flattened Euler sub-steps: t = 0 predictor (Q0 of 5 cells -> Q1),
    t = 1 corrector (Q1 of 5 cells and own Q0 -> Q0)."""
    if t == 0:
        return "Q1", _h(*(x["Q0"] for x in nb), m)
    return "Q0", _h(c["Q0"], *(x["Q1"] for x in nb), m)


def _naive_flat(q0, levels):
    n = len(q0)
    st = [{"Q0": v, "Q1": 0} for v in q0]
    for m in range(1, levels + 1):
        t = (m - 1) & 1
        upd = [_flat_update(t, m, st[i], [st[(i + d) % n] for d in (-2, -1, 0, 1, 2)])
               for i in range(n)]
        for i, (f, v) in enumerate(upd):
            st[i][f] = v
    return [c["Q0"] for c in st]


def _swept_flat(q0, levels, width):
    n, R = len(q0), 2
    cur = [({"Q0": v, "Q1": 0}, 0) for v in q0]
    for k, k_count, off, first, last in _phases(levels, width, R):
        nxt = [None] * n
        for t0 in range(off, off + n, width):
            idx = [(t0 - R + i) % n for i in range(width + 2 * R)]
            st = [dict(cur[g][0]) for g in idx]
            top = [cur[g][1] for g in idx]
            for m in range(first, last + 1):
                lo, hi = sw.sw_phase_interval(k, levels, width, m, R)
                upd = {}
                for o in range(lo, hi):
                    i = o + R
                    assert top[i] == m - 1
                    assert all(top[i + d] in (m - 1, m) for d in (-2, -1, 1, 2))
                    upd[i] = _flat_update((m - 1) & 1, m, st[i], [st[i + d] for d in (-2, -1, 0, 1, 2)])
                for i, (f, v) in upd.items():
                    st[i][f] = v
                    top[i] = m
            for i in range(R, width + R):
                nxt[idx[i]] = (st[i], top[i])
        cur = nxt
    return [c[0]["Q0"] for c in cur]


@pytest.mark.parametrize("n,width", [(8, 4), (16, 8), (32, 8), (48, 16)])
def test_flat_struct_schedule_equals_stepping(n, width):
    rng = random.Random(5 * n + width)
    q0 = [rng.getrandbits(60) for _ in range(n)]
    for steps in sorted({0, 1, 2, 3, rng.randint(1, width)}):
        assert _swept_flat(q0, 2 * steps, width) == _naive_flat(q0, 2 * steps)


@pytest.mark.parametrize("width", [4, 8, 64, 1024])
def test_structural_facts_of_the_paper(width):
    """Sec. 4.1: the Up Triangle ends with two values at the centre after W/2
    sub-steps, and each exchange between neighbouring blocks moves W/2 + 1
    values: a tile of the next phase reads its W cells and one halo cell per
    side, W/2 + 1 of them from each of the two tiles of the previous phase
    that it straddles."""
    half = width // 2
    levels = 5 * half
    lo, hi = sw.sw_phase_interval(1, levels, width, half)
    assert (lo, hi) == (half - 1, half + 1)          # two centre values at level W/2
    for k in range(2, sw.sw_phase_count(levels, width) + 1):
        off_prev = sw.sw_phase_info(k - 1, levels, width)[0]
        off = sw.sw_phase_info(k, levels, width)[0]
        assert (off - off_prev) % width == half       # shifted by W/2
        n = 4 * width
        t0 = off + width                               # any tile of phase k
        reads = set(range(t0 - 1, t0 + width + 1))     # W + 2 cells
        owners = {}
        for c in reads:
            owner = ((c - off_prev) % n) // width     # previous-phase tile holding cell c
            owners[owner] = owners.get(owner, 0) + 1
        assert sorted(owners.values()) == [half + 1, half + 1]
