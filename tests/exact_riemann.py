"""Exact solution of the Riemann problem for the 1D Euler equations (ideal gas).

Independent of the oracle: the star pressure is found by Newton iteration on
the pressure function, and the self-similar solution is sampled from the wave
pattern (textbook exact solver, Toro, "Riemann Solvers and Numerical Methods
for Fluid Dynamics", ch. 4).  Used to pin the Euler oracle on shock tubes.
"""
import math

GAMMA = 1.4


def _f_and_df(p, rho, pk, ak):
    if p > pk:  # shock
        a = 2.0 / ((GAMMA + 1.0) * rho)
        b = (GAMMA - 1.0) / (GAMMA + 1.0) * pk
        q = math.sqrt(a / (p + b))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (b + p))
    # rarefaction
    pr = p / pk
    f = 2.0 * ak / (GAMMA - 1.0) * (pr ** ((GAMMA - 1.0) / (2.0 * GAMMA)) - 1.0)
    df = 1.0 / (rho * ak) * pr ** (-(GAMMA + 1.0) / (2.0 * GAMMA))
    return f, df


def star_state(left, right):
    """(p*, u*, rho*_L, rho*_R) for primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = math.sqrt(GAMMA * pl / rl), math.sqrt(GAMMA * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _f_and_df(p, rl, pl, al)
        fr, dfr = _f_and_df(p, rr, pr, ar)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, 1e-12)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, al)
    fr, _ = _f_and_df(p, rr, pr, ar)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    g = (GAMMA - 1.0) / (GAMMA + 1.0)
    if p > pl:
        rsl = rl * (p / pl + g) / (g * p / pl + 1.0)
    else:
        rsl = rl * (p / pl) ** (1.0 / GAMMA)
    if p > pr:
        rsr = rr * (p / pr + g) / (g * p / pr + 1.0)
    else:
        rsr = rr * (p / pr) ** (1.0 / GAMMA)
    return p, u, rsl, rsr


def sample(left, right, xi):
    """Primitive state (rho, u, p) at similarity coordinate xi = x / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us, rsl, rsr = star_state(left, right)
    al, ar = math.sqrt(GAMMA * pl / rl), math.sqrt(GAMMA * pr / rr)
    if xi <= us:  # left of the contact
        if ps > pl:  # left shock
            sl = ul - al * math.sqrt((GAMMA + 1) / (2 * GAMMA) * ps / pl + (GAMMA - 1) / (2 * GAMMA))
            return (rl, ul, pl) if xi <= sl else (rsl, us, ps)
        head = ul - al
        asl = al * (ps / pl) ** ((GAMMA - 1) / (2 * GAMMA))
        tail = us - asl
        if xi <= head:
            return (rl, ul, pl)
        if xi >= tail:
            return (rsl, us, ps)
        c = 2 / (GAMMA + 1) + (GAMMA - 1) / ((GAMMA + 1) * al) * (ul - xi)
        rho = rl * c ** (2 / (GAMMA - 1))
        u = 2 / (GAMMA + 1) * (al + (GAMMA - 1) / 2 * ul + xi)
        p = pl * c ** (2 * GAMMA / (GAMMA - 1))
        return (rho, u, p)
    if ps > pr:  # right shock
        sr = ur + ar * math.sqrt((GAMMA + 1) / (2 * GAMMA) * ps / pr + (GAMMA - 1) / (2 * GAMMA))
        return (rr, ur, pr) if xi >= sr else (rsr, us, ps)
    head = ur + ar
    asr = ar * (ps / pr) ** ((GAMMA - 1) / (2 * GAMMA))
    tail = us + asr
    if xi >= head:
        return (rr, ur, pr)
    if xi <= tail:
        return (rsr, us, ps)
    c = 2 / (GAMMA + 1) - (GAMMA - 1) / ((GAMMA + 1) * ar) * (ur - xi)
    rho = rr * c ** (2 / (GAMMA - 1))
    u = 2 / (GAMMA + 1) * (-ar + (GAMMA - 1) / 2 * ur + xi)
    p = pr * c ** (2 * GAMMA / (GAMMA - 1))
    return (rho, u, p)


def shock_speed(left, right):
    """Speed of the right-moving shock when p* > p_R."""
    rr, ur, pr = right
    ps, _, _, _ = star_state(left, right)
    ar = math.sqrt(GAMMA * pr / rr)
    return ur + ar * math.sqrt((GAMMA + 1) / (2 * GAMMA) * ps / pr + (GAMMA - 1) / (2 * GAMMA))
