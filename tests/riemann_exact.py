"""Exact solution of the 1D Euler Riemann problem for an ideal gas (the
textbook construction: star pressure from the pressure function by Newton
iteration, then the wave pattern sampled along x/t).  Independent test
infrastructure for the shock-tube pins."""
from __future__ import annotations

import math

import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = p / pk
    return (2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0),
            1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g)))


def star_state(left, right, g=1.4, tol=1e-14):
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum generated")
    p = max(tol, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(tol, p - dp)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, xi, g=1.4):
    """(rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    gm = (g - 1.0) / (g + 1.0)
    out = np.zeros((3, np.size(xi)))
    for k, s in enumerate(np.atleast_1d(xi)):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rs = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                S = ul - cl * math.sqrt((g + 1.0) / (2 * g) * ps / pl + (g - 1.0) / (2 * g))
                out[:, k] = (rl, ul, pl) if s <= S else (rs, us, ps)
            else:  # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / g)
                cs = cl * (ps / pl) ** ((g - 1.0) / (2 * g))
                if s <= ul - cl:
                    out[:, k] = (rl, ul, pl)
                elif s >= us - cs:
                    out[:, k] = (rs, us, ps)
                else:
                    u = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + s)
                    c = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * (ul - s))
                    rho = rl * (c / cl) ** (2.0 / (g - 1.0))
                    out[:, k] = (rho, u, pl * (c / cl) ** (2 * g / (g - 1.0)))
        else:  # right of contact
            if ps > pr:  # right shock
                rs = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                S = ur + cr * math.sqrt((g + 1.0) / (2 * g) * ps / pr + (g - 1.0) / (2 * g))
                out[:, k] = (rr, ur, pr) if s >= S else (rs, us, ps)
            else:  # right rarefaction
                rs = rr * (ps / pr) ** (1.0 / g)
                cs = cr * (ps / pr) ** ((g - 1.0) / (2 * g))
                if s >= ur + cr:
                    out[:, k] = (rr, ur, pr)
                elif s <= us + cs:
                    out[:, k] = (rs, us, ps)
                else:
                    u = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + s)
                    c = 2.0 / (g + 1.0) * (cr - (g - 1.0) / 2.0 * (ur - s))
                    rho = rr * (c / cr) ** (2.0 / (g - 1.0))
                    out[:, k] = (rho, u, pr * (c / cr) ** (2 * g / (g - 1.0)))
    return out


def wave_speeds(left, right, g=1.4):
    """Fastest left- and right-going signal speeds (for the boundary-influence zone)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    sl = ul - cl * (math.sqrt((g + 1.0) / (2 * g) * ps / pl + (g - 1.0) / (2 * g)) if ps > pl else 1.0)
    sr = ur + cr * (math.sqrt((g + 1.0) / (2 * g) * ps / pr + (g - 1.0) / (2 * g)) if ps > pr else 1.0)
    return sl, sr
