"""Lane-level CPU emulation of the heat kernels' register-blocked level sweep
(rows of 64 lanes, kRbC cells per lane, DPP neighbour shifts, ghost lanes,
edge masks, the split between the upward rows and the downward edge row),
written from the kernel's description, with the kernel's constants.  The
tests replay phases of every shape through it and compare with the plain
level-by-level sweep: a wrong mask, margin, split or parity fails there."""
import numpy as np

C, L, OWNED, ROWS_PER_WAVE = 5, 5, 62, 2
PAD = C


def update(l, c, rr, r):
    """The scheme as written (the plain sweep and the oracle)."""
    return c + r * ((rr - c) + (l - c))


def plain_levels(s, w, base, js, r):
    for j in js:
        a = abs(j - 1)
        m = base + j
        src, dst = s[(m & 1) ^ 1], s[m & 1]
        new = [update(src[i - 1], src[i], src[i + 1], r) for i in range(a + 1, w - a + 1)]
        dst[a + 1: w - a + 1] = new


def _block(s, w, base, ja, jz, r, waves):
    wid = jz <= 1
    nl = jz - ja + 1
    a_out = 1 - jz if wid else ja - 1
    t_lo, t_hi = (L - nl, L) if wid else (0, nl)
    jv0 = jz - (L - 1) if wid else ja
    e_lo, e_hi = a_out + 1, w - a_out
    wo = e_hi - e_lo + 1
    qmin = -(-(2 * L + C - 1) // C)
    q = max(-(-wo // C) - OWNED, qmin)
    rows = 1 + -(-q // OWNED)
    if C * q > wo - 1 - 2 * L or rows > waves * ROWS_PER_WAVE:
        return False
    sp = e_lo + C * q
    p0 = (base + jv0) & 1
    lane = np.arange(64)

    def get(slot, idx):
        inside = (idx >= 0) & (idx <= w + 1)
        return np.where(inside, s[slot][np.clip(idx, 0, w + 1)], 1e6 + idx)

    rs = []
    for f in range(rows):
        if f == 1:  # right edge row, lanes downward
            start = e_hi - lane * C + 1
            wr = (lane >= 1) & (lane <= OWNED) & (start + C - 1 >= sp)
        else:
            row = 0 if f == 0 else f - 1
            start = e_lo + OWNED * C * row + (lane - 1) * C
            wr = (lane >= 1) & (lane <= OWNED) & (start < sp)
        start = np.clip(start, -PAD, w + 2 + PAD - C)
        idx = start[:, None] + np.arange(C)[None, :]
        v = np.stack([get(p0, idx), get(p0 ^ 1, idx)])
        rs.append((f, v, idx, wr))
    for t in range(t_lo, t_hi):
        q_w, q_r = t & 1, (t & 1) ^ 1
        frz = L - 1 - t if wid else t
        for f, v, idx, wr in rs:
            src = v[q_r]
            prev_last = np.concatenate([[0.0], src[:-1, C - 1]])
            next_last = np.concatenate([src[1:, C - 1], [0.0]])
            prev_first = np.concatenate([[0.0], src[:-1, 0]])
            next_first = np.concatenate([src[1:, 0], [0.0]])
            below, above = (next_last, prev_first) if f == 1 else (prev_last, next_first)
            ext = np.concatenate([below[:, None], src, above[:, None]], axis=1)
            d = ext[:, 1:] - ext[:, :-1]               # one difference per face
            new = src + r * (d[:, 1:] - d[:, :-1])
            keep = np.zeros((64, C), bool)
            if f == 0:
                keep[0, C - 1] = True
                keep[1, :frz] = True
            elif f == 1:
                keep[0, 0] = True
                if frz:
                    keep[1, C - frz:] = True
            v[q_w] = np.where(keep, v[q_w], new)
    for f, v, idx, wr in rs:
        for lan in np.nonzero(wr)[0]:
            assert np.all((idx[lan] >= e_lo) & (idx[lan] <= e_hi))
            s[p0][idx[lan]] = v[0, lan]
            s[p0 ^ 1][idx[lan]] = v[1, lan]
    return True


def blocked_levels(s, w, base, j_first, j_last, r, waves=4):
    """The kernel's sweep of levels j_first..j_last of one tile phase."""
    jw = min(1, j_last)
    if j_first <= jw:
        sz = (jw - j_first + 1) % L or L
        j = j_first
        while j <= jw:
            if not _block(s, w, base, j, j + sz - 1, r, waves):
                plain_levels(s, w, base, range(j, j + sz), r)
            j += sz
            sz = L
    j = max(2, j_first)
    while j <= j_last:
        jz = min(j + L - 1, j_last)
        if not _block(s, w, base, j, jz, r, waves):
            plain_levels(s, w, base, range(j, jz + 1), r)
        j = jz + 1
