"""Host emulation of the batched persistent launch (no GPU).

The persistent kernel runs work items (phase, tile) of a problem in any order
its completion flags allow, concurrently.  Here every item reads its inputs
when it starts and writes its outputs when it finishes, and the emulator
interleaves starts and finishes at random under exactly the dependency rule
the kernel uses (queried from the library, sw_batch_item_deps).  Any data race
the rule allowed -- a tile reading a cell before its producer wrote it, or a
tile overwriting a working-array cell a slower reader still needed -- changes
the opaque hash result against plain stepping.
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


def _naive(u0, levels):
    n = len(u0)
    u = list(u0)
    for m in range(1, levels + 1):
        u = [_h(u[i - 1], u[i], u[(i + 1) % n], m) for i in range(n)]
    return u


def _emulate(u0, levels, width, seed):
    """Random concurrent interleaving of the batch items of one heat-like problem."""
    rng = random.Random(seed)
    n = len(u0)
    tiles = n // width
    phases = sw.sw_phase_count(levels, width)
    single = 1 if phases == 1 else 0
    item_phases = phases + single
    state = list(u0)
    ws = [[(None, None)] * n, [(None, None)] * n]  # ws[0] written by odd phases
    flags = [0] * tiles
    pending = [(k, t) for k in range(1, item_phases + 1) for t in range(tiles)]
    running = {}  # item -> snapshot
    done = set()

    def ready(k, t):
        deps = sw.sw_batch_item_deps(k, t, tiles, single)
        return all(flags[d] >= k - 1 for d in deps)

    def start(k, t):
        if single and k == 2:
            return ("copy", [ws[0][t * width + i] for i in range(width)])
        off, first, last = sw.sw_phase_info(k, levels, width)
        g0 = off + t * width - 1
        idx = [(g0 + i) % n for i in range(width + 2)]
        if k == 1:
            cells = [[state[g], None] for g in idx]
            top = [0] * (width + 2)
        else:
            src = ws[0] if k % 2 == 0 else ws[1]
            cells = [list(src[g][0]) if src[g][0] is not None else [None, None] for g in idx]
            top = [src[g][1] for g in idx]
        return ("tile", idx, cells, top, first, last)

    def finish(k, t, snap):
        if snap[0] == "copy":
            for i, (sl, top) in enumerate(snap[1]):
                state[t * width + i] = sl[top & 1]
            return
        _, idx, cells, top, first, last = snap
        for m in range(first, last + 1):
            lo, hi = sw.sw_phase_interval(k, levels, width, m)
            new = {}
            for o in range(lo, hi):
                i = o + 1
                assert top[i] == m - 1
                assert top[i - 1] in (m - 1, m) and top[i + 1] in (m - 1, m)
                src = (m - 1) & 1
                assert None not in (cells[i - 1][src], cells[i][src], cells[i + 1][src])
                new[i] = _h(cells[i - 1][src], cells[i][src], cells[i + 1][src], m)
            for i, v in new.items():
                cells[i][m & 1] = v
                top[i] = m
        if k == phases and not single:
            for i in range(1, width + 1):
                state[idx[i]] = cells[i][levels & 1]
        else:
            dst = ws[0] if k % 2 == 1 else ws[1]
            for i in range(1, width + 1):
                dst[idx[i]] = (tuple(cells[i]), top[i])

    while pending or running:
        choices = [("s", it) for it in pending if ready(*it)] + [("f", it) for it in running]
        kind, it = rng.choice(choices)
        if kind == "s":
            pending.remove(it)
            running[it] = start(*it)
        else:
            finish(*it, running.pop(it))
            flags[it[1]] = it[0]
            done.add(it)
    return state


@pytest.mark.parametrize("n,width", [(8, 4), (12, 4), (16, 8), (24, 6), (32, 8), (64, 16), (40, 10)])
def test_any_flag_respecting_interleaving_equals_stepping(n, width):
    rng = random.Random(n * 31 + width)
    u0 = [rng.getrandbits(60) for _ in range(n)]
    h = width // 2
    for levels in sorted({1, 2, h, h + 1, 3 * h + 1, rng.randint(1, 5 * h)}):
        want = _naive(u0, levels)
        for seed in range(3):
            assert _emulate(u0, levels, width, seed) == want, (n, width, levels, seed)


def test_dependency_rule():
    # even phases (offset W/2) wait for tiles t, t+1; odd phases for t-1, t
    assert sw.sw_batch_item_deps(1, 3, 8) == []
    assert sw.sw_batch_item_deps(2, 3, 8) == [3, 4]
    assert sw.sw_batch_item_deps(3, 3, 8) == [2, 3]
    assert sw.sw_batch_item_deps(2, 7, 8) == [7, 0]
    assert sw.sw_batch_item_deps(3, 0, 8) == [7, 0]
    assert sw.sw_batch_item_deps(2, 1, 4, 1) == [0, 1, 2]


def test_emulator_catches_a_weaker_rule(monkeypatch):
    """Dropping either dependency must produce a detectable race."""
    orig = sw.sw_batch_item_deps
    rng = random.Random(1)
    u0 = [rng.getrandbits(60) for _ in range(32)]
    want = _naive(u0, 25)
    for weaker in (lambda k, t, n, s=0: [], lambda k, t, n, s=0: orig(k, t, n, s)[:1],
                   lambda k, t, n, s=0: orig(k, t, n, s)[1:]):
        monkeypatch.setattr(sw, "sw_batch_item_deps", weaker)
        caught = 0
        for seed in range(10):
            try:
                caught += _emulate(u0, 25, 8, seed) != want
            except (AssertionError, TypeError):
                caught += 1
        assert caught >= 5
    monkeypatch.setattr(sw, "sw_batch_item_deps", orig)


def test_item_numbering_is_a_phase_major_bijection(tmp_path):
    """The persistent kernel resolves a ticket number through the sorted
    problem table alone (two binary searches, no per-phase table).  A host
    build of that lookup and of the planner, over 300 random problem lists,
    must map the item numbers one to one onto (problem, phase, tile) with
    phases non-decreasing."""
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    csrc = os.path.join(os.path.dirname(here), "paper_1811_08282_amd", "csrc")
    exe = str(tmp_path / "batch_table_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-I", csrc, "-o", exe,
                    os.path.join(here, "batch_table_check.cpp")], check=True)
    out = subprocess.run([exe, "300"], check=True, capture_output=True, text=True)
    assert out.stdout.startswith("ok 300")
