"""Seeded synthetic inputs for the D2V16 MRT-FD step.

This module builds the initial fields (rho, u_x, u_y, T on every node) and the
run parameters of the paper's test problems and of the larger synthetic
workloads.  It holds none of the method's arithmetic: no moments, equilibria,
collision or fluxes -- only grids, gas states (ideal gas, P = rho T with
R = 1, gamma = (b + 2) / b as in Sec. II) and seeded random draws.  Both the
GPU path and the CPU oracle consume what it returns.

A case is a dict::

    {"name": str, "params": {...}, "rho": (ny, nx), "ux": ..., "uy": ..., "T": ...,
     "nsteps": int}

``params`` carries nx, ny, dx, dy, dt, eta0, s[16], b, limiter, correction,
precision and bc[4] (x-lo, x-hi, y-lo, y-hi), each bc a dict
``{"kind": "periodic" | "equilibrium" | "outflow" | "wall", "state": (rho, ux, uy, T)}``.
"""
from __future__ import annotations

import math

import numpy as np

ETA0 = 2.5  # extra-DOF parameter of the |v| = 1 group (Appendix)


def b_of_gamma(gamma: float) -> float:
    """gamma = (b + 2) / b  (Sec. II)."""
    return 2.0 / (gamma - 1.0)


def bc(kind: str, rho=1.0, ux=0.0, uy=0.0, T=1.0) -> dict:
    return {"kind": kind, "state": (float(rho), float(ux), float(uy), float(T))}


def make_params(nx, ny, dx, dy, dt, s, b, bcs, limiter="mc", correction=True,
                precision="fp64") -> dict:
    s = [float(v) for v in s]
    assert len(s) == 16 and len(bcs) == 4
    return {"nx": int(nx), "ny": int(ny), "dx": float(dx), "dy": float(dy), "dt": float(dt),
            "eta0": ETA0, "s": s, "b": float(b), "limiter": limiter,
            "correction": bool(correction), "precision": precision, "bc": list(bcs)}


def rates(conserved, viscous, heat, other):
    """s_1..4 (no effect), s_5..7 (viscous), s_8..9 (heat flux), s_10..16."""
    return [conserved] * 4 + [viscous] * 3 + [heat] * 2 + [other] * 7


def _case(name, params, rho, ux, uy, T, nsteps):
    ny, nx = params["ny"], params["nx"]
    f = lambda a: np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), (ny, nx)))
    return {"name": name, "params": params, "rho": f(rho), "ux": f(ux), "uy": f(uy), "T": f(T),
            "nsteps": int(nsteps)}


def cell_centres(n: int, d: float, origin: float = 0.0) -> np.ndarray:
    return origin + (np.arange(n) + 0.5) * d


# --------------------------------------------------------------------------
# Shock tubes (Sec. IV-A/B style problems)

def riemann_1d(left, right, gamma, nx, ny=1, length=1.0, x0=0.5, cfl=0.1, s_cons=1e4,
               s_nc=1e3, s=None, limiter="minmod", t_end=None, nsteps=None, precision="fp64",
               name="riemann"):
    """Two-state Riemann problem in x, equilibrium ghosts at the initial states,
    periodic in y.  ``left``/``right`` are (rho, u, p)."""
    b = b_of_gamma(gamma)
    dx = length / nx
    dt = dx * cfl / 6.0            # Courant number cfl on the fastest speed |v| = 6
    rl, ul, pl = left
    rr, ur, pr = right
    Tl, Tr = pl / rl, pr / rr
    x = cell_centres(nx, dx)
    isl = (x < x0)[None, :].repeat(ny, 0)
    rho = np.where(isl, rl, rr)
    ux = np.where(isl, ul, ur)
    T = np.where(isl, Tl, Tr)
    if s is None:
        s = [s_cons] * 4 + [s_nc] * 12
    bcs = [bc("equilibrium", rl, ul, 0.0, Tl), bc("equilibrium", rr, ur, 0.0, Tr),
           bc("periodic"), bc("periodic")]
    if nsteps is None:
        nsteps = int(round(t_end / dt))
    p = make_params(nx, ny, dx, dx, dt, s, b, bcs, limiter=limiter, precision=precision)
    return _case(name, p, rho, ux, 0.0, T, nsteps)


def sod(limiter="minmod", nx=400, ny=1, precision="fp64"):
    """Sod tube: (1, 0, 1) | (0.125, 0, 0.1), gamma = 1.4, dx = 1/400,
    dt = dx*0.1/6, t = 0.15 (3600 steps), s = 1e4 conserved / 1e3 others."""
    return riemann_1d((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, nx, ny=ny, cfl=0.1,
                      s_cons=1e4, s_nc=1e3, limiter=limiter, t_end=0.15,
                      precision=precision, name="sod")


# --------------------------------------------------------------------------
# Thermal Couette flow (Sec. IV-C, rotated: walls at y = 0 and y = 1)

def couette(pr=1.0, gamma=1.4, nx=4, ny=200, u0=0.2, s5=50.0, s_other=None, T_wall=1.0,
            dt_over_dy=1.0 / 12.0, start="rest", precision="fp64", limiter="mc",
            correction=True):
    """Walls on the first and last grid rows (y_j = j / (ny - 1)); the upper
    wall moves with u_x = u0, both walls at T_wall; periodic in x.
    s_5..7 = s5, s_8..9 = Pr s5, all other rates s5 unless given.
    ``start="rest"`` begins from rho = 1, u = 0, T = 1; ``start="profile"``
    begins from the linear velocity profile (steady-state tests only)."""
    b = b_of_gamma(gamma)
    dy = 1.0 / (ny - 1)
    dx = dy
    dt = dy * dt_over_dy
    if s_other is None:
        # rates of the higher moments equal to s_5: the linearised model is
        # unstable at short wavelengths when they exceed s_5 by much
        s_other = s5
    s = rates(s_other, s5, pr * s5, s_other)
    bcs = [bc("periodic"), bc("periodic"), bc("wall", 1.0, 0.0, 0.0, T_wall),
           bc("wall", 1.0, u0, 0.0, T_wall)]
    y = np.arange(ny) * dy
    ux = np.zeros((ny, nx))
    if start == "profile":
        ux = np.repeat((u0 * y)[:, None], nx, 1)
    p = make_params(nx, ny, dx, dy, dt, s, b, bcs, limiter=limiter, correction=correction,
                    precision=precision)
    return _case(f"couette_pr{pr}_g{gamma}", p, 1.0, ux, 0.0, T_wall, 0)


def couette_analytic(y, pr, gamma, u0=0.2, T1=1.0, T2=1.0, H=1.0):
    """u = u0 y / H; T = T1 + (T2 - T1) y/H + (mu / 2 lambda) u0^2 (y/H)(1 - y/H)
    with mu / lambda = Pr / c_p, c_p = (b + 2) / 2 (Sec. II and IV-C)."""
    b = b_of_gamma(gamma)
    cp = (b + 2.0) / 2.0
    eta = np.asarray(y) / H
    return u0 * eta, T1 + (T2 - T1) * eta + 0.5 * pr / cp * u0 ** 2 * eta * (1.0 - eta)


# --------------------------------------------------------------------------
# Shock from a heavy medium into a light one (Sec. V, generalised)

def normal_shock(rho1, p1, mach, gamma):
    """Rankine-Hugoniot post-shock state for a shock moving at Mach ``mach``
    into gas at rest: returns (rho2, u2, p2, shock speed)."""
    g = gamma
    c1 = math.sqrt(g * p1 / rho1)
    W = mach * c1
    rho2 = rho1 * (g + 1) * mach ** 2 / ((g - 1) * mach ** 2 + 2)
    p2 = p1 * (1 + 2 * g / (g + 1) * (mach ** 2 - 1))
    u2 = W * (1 - rho1 / rho2)
    return rho2, u2, p2, W


def shock_interface(nx=4096, ny=1024, gamma=1.4, mach=2.0, rho_heavy=5.0, rho_light=1.0,
                    p0=1.0, x_shock=0.94, x_int=1.0, amp=0.05, dt=1e-5, nsteps=2000,
                    precision="fp64", limiter="mc"):
    """Domain [0, nx/ny] x [0, 1], dx = dy = 1/ny, cell-centred.  A Mach-2
    shock (post-shock state for x < x_shock) runs into heavy gas at rest that
    meets light gas at equal pressure across x_I(y) = x_int + amp sin(2 pi y).
    Inflow = equilibrium ghosts at the post-shock state, outflow on the right,
    periodic in y.  Rates as in Sec. V: s_5..7 = 5e4, others 1e5."""
    b = b_of_gamma(gamma)
    d = 1.0 / ny
    r2, u2, p2, _ = normal_shock(rho_heavy, p0, mach, gamma)
    x = cell_centres(nx, d)[None, :]
    y = cell_centres(ny, d)[:, None]
    xi = x_int + amp * np.sin(2.0 * math.pi * y)
    rho = np.where(x > xi, rho_light, rho_heavy) * np.ones((ny, nx))
    T = np.where(x > xi, p0 / rho_light, p0 / rho_heavy) * np.ones((ny, nx))
    ux = np.zeros((ny, nx))
    post = (x < x_shock) * np.ones((ny, nx), bool)
    rho = np.where(post, r2, rho)
    T = np.where(post, p2 / r2, T)
    ux = np.where(post, u2, ux)
    s = rates(1e5, 5e4, 1e5, 1e5)
    bcs = [bc("equilibrium", r2, u2, 0.0, p2 / r2), bc("outflow"), bc("periodic"), bc("periodic")]
    p = make_params(nx, ny, d, d, dt, s, b, bcs, limiter=limiter, precision=precision)
    return _case(f"shock_interface_{nx}x{ny}", p, rho, ux, 0.0, T, nsteps)


def paper_heavy_light(precision="fp64"):
    """The paper's own run (Sec. V): [0, 1.2] x [0, 0.01], 1200 x 10 cells,
    gamma = 2, states s = (1.5, 2/3, 0, p = 7/3), h = (1, 0, 0, 1),
    l = (0.5, 0, 0, 1); shock at 0.24, interface at 0.4; t = 0.3."""
    nx, ny, d = 1200, 10, 0.001
    gamma = 2.0
    b = b_of_gamma(gamma)
    x = cell_centres(nx, d)[None, :] * np.ones((ny, 1))
    rs, us, ps = 1.5, 2.0 / 3.0, 7.0 / 3.0
    rho = np.where(x < 0.24, rs, np.where(x < 0.4, 1.0, 0.5))
    ux = np.where(x < 0.24, us, 0.0)
    T = np.where(x < 0.24, ps / rs, np.where(x < 0.4, 1.0, 2.0))
    s = rates(1e5, 5e4, 1e5, 1e5)
    bcs = [bc("equilibrium", rs, us, 0.0, ps / rs), bc("outflow"), bc("periodic"), bc("periodic")]
    p = make_params(nx, ny, d, d, 1e-5, s, b, bcs, precision=precision)
    return _case("paper_heavy_light", p, rho, ux, 0.0, T, 30000)


# --------------------------------------------------------------------------
# Batched Riemann instances (512 by default)

# Stability envelope of the 16-velocity model with the rates below: states
# are redrawn until the temperature and the pressure ratios across the
# problem stay within bounds and every initial state is subsonic (strong
# shocks, cold regions and supersonic states beyond these drive some node to
# a negative temperature, in the oracle and on the GPU alike).  A screen is
# (temperature ratio, pressure ratio, Mach number) bounds.  The batch takes
# the widest screen found under which none of its 512 draws has a node with
# rho <= 0, T <= 0 or a non-finite value after any of its 1000 steps in the
# oracle: temperature ratio 5, pressure ratio 7, subsonic (291 redraws).
# tests/golden/make_screen_envelope.py counts the failing draws under this
# and twelve other screens: every wider one tried has some (a temperature
# ratio of 20 alone: 58 of 512).  The four-quadrant requests of the served
# stream keep ratios of 5.
SCREEN_RATIO = 5.0
SCREEN_MACH = 1.0
SCREEN = (SCREEN_RATIO, 7.0, SCREEN_MACH)


def riemann_batch(n=512, seed=13054736, nsteps=1000, precision="fp32", screen=SCREEN):
    """Independent two-state Riemann problems with log-uniform Nx in
    [128, 4096], Ny in [1, 256]; rho, p ~ U[0.1, 10], u ~ U[-0.5, 0.5],
    gamma ~ U[1.1, 1.67]; states (and gamma) are redrawn while the
    temperature ratio, the pressure ratio or a side's Mach number exceeds the
    screen's bounds, then rescaled to T_max = 1
    (p /= T_ref, u /= sqrt(T_ref)).  dt = 0.01 dx, dt*s = 0.5 (s_5..7) and 1
    (the others).  Returns (cases, redraws)."""
    t_max, p_max, m_max = screen
    rng = np.random.default_rng(seed)
    cases = []
    redraws = 0
    for k in range(n):
        nx = int(round(math.exp(rng.uniform(math.log(128), math.log(4096)))))
        ny = int(round(math.exp(rng.uniform(0.0, math.log(256)))))
        while True:
            rl, rr = rng.uniform(0.1, 10.0, 2)
            pl, pr = rng.uniform(0.1, 10.0, 2)
            ul, ur = rng.uniform(-0.5, 0.5, 2)
            gamma = rng.uniform(1.1, 1.67)
            Tl, Tr = pl / rl, pr / rr
            mach = max(abs(ul) / math.sqrt(gamma * Tl), abs(ur) / math.sqrt(gamma * Tr))
            if max(Tl, Tr) / min(Tl, Tr) <= t_max and max(pl, pr) / min(pl, pr) <= p_max and mach <= m_max:
                break
            redraws += 1
        Tref = max(Tl, Tr)
        pl, pr = pl / Tref, pr / Tref
        ul, ur = ul / math.sqrt(Tref), ur / math.sqrt(Tref)
        dx = 1.0 / nx
        dt = 0.06 * dx / 6.0
        s = rates(1.0 / dt, 0.5 / dt, 1.0 / dt, 1.0 / dt)
        c = riemann_1d((rl, ul, pl), (rr, ur, pr), gamma, nx, ny=ny, s=s, limiter="mc",
                       nsteps=nsteps, precision=precision, name=f"riemann_{k}")
        c["params"]["dt"] = dt
        cases.append(c)
    return cases, redraws


# --------------------------------------------------------------------------
# Served stream of requests.  A request is a compact spec (parameters plus a
# piecewise-constant initial state) so that its fields can be built where
# they are used (numpy on the host, torch on the device).

def _quadrant_spec(rng, nx, ny, nsteps, precision, name):
    while True:
        rho = rng.uniform(0.25, 4.0, 4)
        p = rng.uniform(0.25, 4.0, 4)
        u = rng.uniform(-0.3, 0.3, 4)
        v = rng.uniform(-0.3, 0.3, 4)
        T = p / rho
        mach = (np.hypot(u, v) / np.sqrt(1.4 * T)).max()
        if T.max() / T.min() <= SCREEN_RATIO and p.max() / p.min() <= SCREEN_RATIO and mach <= SCREEN_MACH:
            break
    Tref = T.max()
    T = T / Tref
    u, v = u / math.sqrt(Tref), v / math.sqrt(Tref)
    gamma = 1.4
    dx, dy = 1.0 / nx, 1.0 / ny
    dt = 0.06 * min(dx, dy) / 6.0
    s = rates(1.0 / dt, 0.5 / dt, 1.0 / dt, 1.0 / dt)
    bcs = [bc("outflow")] * 4
    prm = make_params(nx, ny, dx, dy, dt, s, b_of_gamma(gamma), bcs, precision=precision)
    # quadrants 0: x < 1/2, y < 1/2; 1: x >= 1/2, y < 1/2; 2: x < 1/2, y >= 1/2; 3: both >= 1/2
    return {"name": name, "kind": "quadrant", "params": prm, "nsteps": int(nsteps),
            "quad": {"rho": rho.tolist(), "ux": u.tolist(), "uy": v.tolist(), "T": T.tolist()}}


def _couette_spec(rng, nx, ny, nsteps, precision, name):
    pr = rng.uniform(0.3, 3.0)
    c = couette(pr=pr, gamma=1.4, nx=nx, ny=ny, precision=precision)
    return {"name": name, "kind": "couette", "params": c["params"], "nsteps": int(nsteps),
            "uniform": {"rho": 1.0, "ux": 0.0, "uy": 0.0, "T": 1.0}, "pr": pr}


def serve_request(rng, k, log_lo=64, log_hi=2048):
    """One request: half Riemann quadrant problems (outflow on all sides),
    half thermal Couette flows with Pr ~ U[0.3, 3]; grid sides log-uniform in
    [log_lo, log_hi]; steps ~ U{200..5000}; FP32 or FP64 storage."""
    kind = "quadrant" if rng.uniform() < 0.5 else "couette"
    nx = int(round(math.exp(rng.uniform(math.log(log_lo), math.log(log_hi)))))
    ny = int(round(math.exp(rng.uniform(math.log(log_lo), math.log(log_hi)))))
    nsteps = int(rng.integers(200, 5001))
    precision = "fp32" if rng.uniform() < 0.5 else "fp64"
    if kind == "quadrant":
        return _quadrant_spec(rng, nx, ny, nsteps, precision, f"req{k}_quadrant")
    return _couette_spec(rng, nx, ny, nsteps, precision, f"req{k}_couette")


def materialize(spec, xp=np, **kw):
    """(rho, ux, uy, T) of a request spec as (ny, nx) float64 arrays of the
    array module xp (numpy, or torch with device=... in kw)."""
    prm = spec["params"]
    nx, ny = prm["nx"], prm["ny"]
    if "uniform" in spec:
        return tuple(xp.full((ny, nx), float(spec["uniform"][k]), dtype=xp.float64, **kw)
                     for k in ("rho", "ux", "uy", "T"))
    xi = (xp.arange(nx, dtype=xp.float64, **kw) + 0.5) * prm["dx"]
    yi = (xp.arange(ny, dtype=xp.float64, **kw) + 0.5) * prm["dy"]
    east = (xi >= 0.5).reshape(1, nx)
    north = (yi >= 0.5).reshape(ny, 1)
    if xp is np:
        qidx = east.astype(np.int64) + 2 * north.astype(np.int64)
        table = lambda v: np.asarray(v, dtype=np.float64)
    else:
        qidx = east.long() + 2 * north.long()
        table = lambda v: xp.tensor(v, dtype=xp.float64, **kw)
    return tuple(table(spec["quad"][k])[qidx].contiguous() if xp is not np else table(spec["quad"][k])[qidx]
                 for k in ("rho", "ux", "uy", "T"))


def spec_case(spec):
    """A request spec as an ordinary case dict (host fields)."""
    r, u, v, T = materialize(spec)
    return _case(spec["name"], spec["params"], r, u, v, T, spec["nsteps"])


def serve_stream(rate=200.0, duration=60.0, seed=13054737, log_lo=64, log_hi=2048,
                 max_requests=None):
    """Poisson arrivals at `rate` per second for `duration` seconds; returns a
    list of (arrival_time_s, spec)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration or (max_requests is not None and len(out) >= max_requests):
            break
        out.append((t, serve_request(rng, len(out), log_lo, log_hi)))
    return out


# --------------------------------------------------------------------------
# Small random cases for parity tests

def random_smooth(nx, ny, seed=0, bcs=None, limiter="mc", precision="fp64", dt_cfl=0.3,
                  amp=0.2, s_visc=40.0, s_heat=30.0, s_other=60.0, gamma=1.4,
                  correction=True, nsteps=10, jumps=False):
    """Random smooth (sum of a few Fourier modes) rho, u, T fields with an
    optional discontinuity; any boundary kinds."""
    rng = np.random.default_rng(seed)
    d = 1.0 / max(nx, ny, 8)
    x = np.arange(nx)[None, :] * d
    y = np.arange(ny)[:, None] * d

    def field(base, a):
        v = np.full((ny, nx), base)
        for _ in range(3):
            kx, ky = rng.integers(1, 4, 2)
            ph = rng.uniform(0, 2 * math.pi)
            v = v + a * rng.uniform(-1, 1) * np.sin(2 * math.pi * (kx * x + ky * y) + ph)
        return v

    rho = field(1.0, amp / 3)
    ux = field(0.0, amp / 2)
    uy = field(0.0, amp / 2)
    T = field(1.0, amp / 3)
    if jumps:
        cut = (x + 0.3 * y > 0.45 * nx * d)
        rho = np.where(cut, rho * 0.5, rho)
        T = np.where(cut, T * 0.8, T)
    if bcs is None:
        bcs = [bc("periodic")] * 4
    dt = dt_cfl * d / 6.0
    s = rates(1e3, s_visc, s_heat, s_other)
    prm = make_params(nx, ny, d, d, dt, s, b_of_gamma(gamma), bcs, limiter=limiter,
                      correction=correction, precision=precision)
    return _case(f"random_{nx}x{ny}_s{seed}", prm, rho, ux, uy, T, nsteps)
