"""Exact solution of the 1D Riemann problem for the Euler equations of an
ideal gas (textbook: Newton/bracketing on the star pressure, then sampling of
the self-similar fan).  Independent of the oracle; used to pin shock-tube runs.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _f_side(p, rho, pk, c, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(left, right, gamma):
    """(p*, u*) for left/right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum generated")
    fun = lambda p: _f_side(p, rl, pl, cl, g) + _f_side(p, rr, pr, cr, g) + (ur - ul)
    hi = max(pl, pr)
    while fun(hi) < 0:
        hi *= 2.0
    ps = brentq(fun, 1e-14, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (_f_side(ps, rr, pr, cr, g) - _f_side(ps, rl, pl, cl, g))
    return ps, us


def sample(left, right, gamma, xi):
    """(rho, u, p) at similarity coordinates xi = (x - x0) / t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, gamma)
    gm = (g - 1.0) / (g + 1.0)
    out = np.zeros((3, len(xi)))
    for n, s in enumerate(np.asarray(xi, dtype=float)):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    w = (rl, ul, pl)
                else:
                    w = (rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps)
            else:  # left rarefaction
                shl = ul - cl
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - csl
                if s <= shl:
                    w = (rl, ul, pl)
                elif s >= stl:
                    w = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    u = 2.0 / (g + 1) * (cl + (g - 1) / 2.0 * ul + s)
                    c = 2.0 / (g + 1) * (cl + (g - 1) / 2.0 * (ul - s))
                    rho = rl * (c / cl) ** (2.0 / (g - 1))
                    w = (rho, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:  # right of contact
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    w = (rr, ur, pr)
                else:
                    w = (rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps)
            else:  # right rarefaction
                shr = ur + cr
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                str_ = us + csr
                if s >= shr:
                    w = (rr, ur, pr)
                elif s <= str_:
                    w = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    u = 2.0 / (g + 1) * (-cr + (g - 1) / 2.0 * ur + s)
                    c = 2.0 / (g + 1) * (cr - (g - 1) / 2.0 * (ur - s))
                    rho = rr * (c / cr) ** (2.0 / (g - 1))
                    w = (rho, u, pr * (c / cr) ** (2 * g / (g - 1)))
        out[:, n] = w
    return out


def shock_speed_right(left, right, gamma):
    rr, ur, pr = right
    g = gamma
    ps, _ = star_state(left, right, gamma)
    cr = math.sqrt(g * pr / rr)
    return ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
