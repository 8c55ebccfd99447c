"""Exact solution of the 1D Riemann problem for an ideal gas (the classical
construction: pressure function of the two non-linear waves, Newton iteration
for the star pressure, then sampling of the self-similar solution).  Used as
an independent reference for the hydro oracle's shock-tube check."""
import math

import numpy as np


def _fk(p, rk, pk, g):
    ck = math.sqrt(g * pk / rk)
    if p > pk:  # shock
        a = 2.0 / ((g + 1.0) * rk)
        b = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(a / (p + b))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + b))
    # rarefaction
    e = (g - 1.0) / (2.0 * g)
    f = 2.0 * ck / (g - 1.0) * ((p / pk) ** e - 1.0)
    return f, (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rk * ck)


def star_state(rl, ul, pl, rr, ur, pr, g=1.4):
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _fk(p, rl, pl, g)
        fr, dr = _fk(p, rr, pr, g)
        pn = max(1e-10, p - (fl + fr + ur - ul) / (dl + dr))
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, g)
    fr, _ = _fk(p, rr, pr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(x, t, x0, left, right, g=1.4):
    """Density, velocity and pressure at positions x (array) and time t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    out = np.zeros((3, len(x)))
    for n, xx in enumerate(x):
        s = (xx - x0) / t
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    w = (rl, ul, pl)
                else:
                    r = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
                    w = (r, us, ps)
            else:
                shl = ul - cl
                cs_ = cl * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - cs_
                if s <= shl:
                    w = (rl, ul, pl)
                elif s >= stl:
                    w = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    r = rl * (c / cl) ** (2 / (g - 1))
                    w = (r, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    w = (rr, ur, pr)
                else:
                    r = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
                    w = (r, us, ps)
            else:
                shr = ur + cr
                cs_ = cr * (ps / pr) ** ((g - 1) / (2 * g))
                str_ = us + cs_
                if s >= shr:
                    w = (rr, ur, pr)
                elif s <= str_:
                    w = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    r = rr * (c / cr) ** (2 / (g - 1))
                    w = (r, u, pr * (c / cr) ** (2 * g / (g - 1)))
        out[:, n] = w
    return out
