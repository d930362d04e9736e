"""Helpers shared by the GPU parity tests: error measures and oracle windows.

Error definitions (relative):  L1 = sum|q - q_o| / sum|q_o|,
Linf = max|q - q_o| / max|q_o| for rho and T.  For the velocity components
the denominators are those of the reference flow speed |u_o| (both
components together): sum|u_o| for L1 and max|u_o| for Linf, so that a
component that is zero everywhere (one-dimensional flows) is not divided by
zero and a slow flow is not measured against its sound speed; only a flow
slower than 1e-3 of the sound speed sqrt(gamma T_ref) everywhere falls back
to that sound speed.
"""
from __future__ import annotations

import math

import numpy as np

TOL = {"fp64": 1e-11, "fp32": 2e-5}
SLOW_FLOW = 1e-3


def velocity_scale(ux_o, uy_o, T_o, gamma=1.4):
    """(L1 denominator, Linf denominator, name) of the velocity errors."""
    speed = np.hypot(np.asarray(ux_o), np.asarray(uy_o))
    cs = math.sqrt(gamma * float(np.max(np.abs(T_o))))
    if speed.max() >= SLOW_FLOW * cs:
        return float(speed.sum()), float(speed.max()), "flow speed"
    return cs * speed.size, cs, "sound speed"


def rel_errors(gpu, orc, gamma=1.4):
    """gpu, orc: (rho, ux, uy, T) tuples -> dict of (L1, Linf) per field."""
    den_u1, den_uinf, _ = velocity_scale(orc[1], orc[2], orc[3], gamma)
    out = {}
    for name, a, b in zip(("rho", "ux", "uy", "T"), gpu, orc):
        a = np.asarray(a)
        b = np.asarray(b)
        diff = np.abs(a - b)
        if name in ("ux", "uy"):
            den_1, den_inf = den_u1, den_uinf
        else:
            den_inf = np.abs(b).max()
            den_1 = np.abs(b).sum()
        out[name] = (diff.sum() / den_1, diff.max() / den_inf)
    return out


def assert_parity(gpu, orc, tol, gamma=1.4, what=""):
    errs = rel_errors(gpu, orc, gamma)
    worst = max(max(v) for v in errs.values())
    assert np.all(np.isfinite(np.concatenate([np.ravel(g) for g in gpu]))), f"{what}: non-finite GPU output"
    assert worst <= tol, f"{what}: errors {errs} exceed {tol}"
    return errs


def f_rel(fg, fo):
    return float(np.abs(fg - fo).max() / np.abs(fo).max())


def window_params(params, x0, nxw, y0, nyw, keep_x_lo, keep_x_hi):
    """Parameters of an (nyw, nxw) sub-window; sides that coincide with the
    real domain edge keep their boundary, the others get outflow (their
    influence is confined to a margin the caller excludes)."""
    p = dict(params)
    p["nx"], p["ny"] = nxw, nyw
    bc = [dict(b) for b in params["bc"]]
    p["bc"] = [bc[0] if keep_x_lo else {"kind": "outflow", "state": (1.0, 0.0, 0.0, 1.0)},
               bc[1] if keep_x_hi else {"kind": "outflow", "state": (1.0, 0.0, 0.0, 1.0)},
               {"kind": "outflow", "state": (1.0, 0.0, 0.0, 1.0)},
               {"kind": "outflow", "state": (1.0, 0.0, 0.0, 1.0)}]
    return p
