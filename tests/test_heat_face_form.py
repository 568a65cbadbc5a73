"""The heat kernels' register-blocked sweep evaluates the FTCS update with
one difference per face instead of two per cell:

    scheme:  u' = u + r * ((u_R - u) + (u_L - u))
    kernel:  d_R = u_R - u,  d_L = u - u_L  (the left cell's d_R)
             u' = u + r * (d_R - d_L)

IEEE subtraction is sign-symmetric, so u_L - u == -(u - u_L) whenever the
difference is not zero, and a + (-b) == a - b exactly.  The only case where
the two sums differ is a signed zero (u_L == u gives +0 in the scheme but
-0 in the kernel's negated face); it needs u == +0 and u_R == -0, where both
forms then give u' = +0.  This test checks the claim bit for bit on triples
built from signed zeros, subnormals, equal neighbours and ordinary values,
in binary64 and in binary32 with the Kahan-compensated update."""
import itertools

import numpy as np


def _specials(dt):
    f = np.finfo(dt)
    base = [0.0, -0.0, f.tiny, -f.tiny, f.tiny * 2 ** -10, -f.tiny * 2 ** -3, 1.0, -1.0,
            1.0 + f.eps, 0.5, 3.0, -2.5, 1e-30 if dt == np.float64 else 1e-20, 7.25e3]
    return np.array(base, dtype=dt)


def _scheme(l, c, r_, r):
    return c + r * ((r_ - c) + (l - c))


def _kernel(l, c, r_, r):
    d_right = r_ - c
    d_left = c - l
    return c + r * (d_right - d_left)


def _kahan(s, c, comp, r):
    d = r * s
    y = d - comp
    t = c + y
    return t, (t - c) - y


def test_face_form_bitwise_binary64_and_binary32():
    for dt, r in ((np.float64, np.float64(0.25)), (np.float64, np.float64(0.3)),
                  (np.float32, np.float32(0.25)), (np.float32, np.float32(0.3))):
        vals = _specials(dt)
        rng = np.random.default_rng(5)
        extra = rng.standard_normal(40).astype(dt) * dt(10.0) ** rng.integers(-30, 30, 40).astype(dt)
        vals = np.concatenate([vals, extra])
        l, c, rr = (a.ravel() for a in np.meshgrid(vals, vals, vals, indexing="ij"))
        with np.errstate(all="ignore"):
            want = _scheme(l, c, rr, r)
            got = _kernel(l, c, rr, r)
        assert np.array_equal(want.view(np.uint64 if dt == np.float64 else np.uint32),
                              got.view(np.uint64 if dt == np.float64 else np.uint32))
        if dt == np.float32:
            for comp0 in (dt(0.0), dt(-0.0), dt(1e-8), dt(-3e-9)):
                comp = np.full_like(c, comp0)
                with np.errstate(all="ignore"):
                    s_scheme = (rr - c) + (l - c)
                    s_kernel = (rr - c) - (c - l)
                    u1, k1 = _kahan(s_scheme, c, comp, r)
                    u2, k2 = _kahan(s_kernel, c, comp, r)
                assert np.array_equal(u1.view(np.uint32), u2.view(np.uint32))
                assert np.array_equal(k1.view(np.uint32), k2.view(np.uint32))


def test_face_form_differs_only_in_the_sign_of_a_zero_sum():
    """The intermediate sums do differ (+0 against -0) on the signed-zero
    triple the docstring names; the update hides it."""
    l, c, rr = np.float64(0.0), np.float64(0.0), np.float64(-0.0)
    s_scheme = (rr - c) + (l - c)
    s_kernel = (rr - c) - (c - l)
    assert np.signbit(s_kernel) != np.signbit(s_scheme)
    assert np.array_equal(np.array([_scheme(l, c, rr, 0.25)]).view(np.uint64),
                          np.array([_kernel(l, c, rr, 0.25)]).view(np.uint64))
