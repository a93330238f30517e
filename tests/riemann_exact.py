"""Exact solution of the 1D Euler Riemann problem (ideal gas), written from the
standard construction: Newton iteration for the star pressure on the sum of the
two wave functions, then sampling of the self-similar fan.  Test helper only."""
import numpy as np


def _wave(p, rk, pk, ck, g):
    if p > pk:   # shock
        A = 2.0 / ((g + 1.0) * rk)
        B = (g - 1.0) / (g + 1.0) * pk
        s = np.sqrt(A / (p + B))
        f = (p - pk) * s
        df = s * (1.0 - 0.5 * (p - pk) / (B + p))
    else:        # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rk * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(L, R, g=1.4):
    rl, ul, pl = L
    rr, ur, pr = R
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    p = max(1e-10, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(200):
        fl, dfl = _wave(p, rl, pl, cl, g)
        fr, dfr = _wave(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _wave(p, rl, pl, cl, g)
    fr, _ = _wave(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(L, R, s, g=1.4):
    """(rho, u, p) at similarity coordinate s = (x - x0)/t."""
    rl, ul, pl = L
    rr, ur, pr = R
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    ps, us = star_state(L, R, g)
    if s <= us:   # left of contact
        if ps > pl:
            rs = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
            sl = ul - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
            return (rl, ul, pl) if s <= sl else (rs, us, ps)
        rs = rl * (ps / pl) ** (1 / g)
        cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
        if s <= ul - cl:
            return (rl, ul, pl)
        if s >= us - cs:
            return (rs, us, ps)
        u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
        c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
        r = rl * (c / cl) ** (2 / (g - 1))
        return (r, u, pl * (c / cl) ** (2 * g / (g - 1)))
    if ps > pr:
        rs = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
        sr = ur + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
        return (rr, ur, pr) if s >= sr else (rs, us, ps)
    rs = rr * (ps / pr) ** (1 / g)
    cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
    if s >= ur + cr:
        return (rr, ur, pr)
    if s <= us + cs:
        return (rs, us, ps)
    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
    r = rr * (c / cr) ** (2 / (g - 1))
    return (r, u, pr * (c / cr) ** (2 * g / (g - 1)))


def density_profile(L, R, x, t, x0=0.5, g=1.4):
    return np.array([sample(L, R, (xx - x0) / t, g)[0] for xx in np.ravel(x)]).reshape(np.shape(x))
