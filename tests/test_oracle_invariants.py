"""Invariants the oracle's full step must satisfy (Sec. II-III).

* a uniform equilibrium state is a fixed point, also between NEE walls that
  move along themselves at the fluid's velocity and temperature (the wall
  node then equals its neighbour; a wall that takes a wrong velocity
  component or sign, a wrong temperature or its nominal density moves it);
* on a periodic grid mass, momentum and energy (rows 1..4 of M) are conserved
  to round-off (the collision leaves them untouched, the fluxes telescope);
* a 90 degree rotation and a mirror of the initial state rotate / mirror the
  solution (catches any x/y or index mix-up in the split fluxes);
* an nx x 1 run equals every row of an nx x 8 run with y-uniform data;
* outflow and equilibrium boundaries do not disturb nodes the waves have not
  reached (domain of dependence of the explicit stencil);
* one step with an outflow or equilibrium side equals one step on a grid
  extended by four lines that hold what the ghosts stand for (copies of the
  last line; the side's equilibrium), on the original nodes: the stencil
  reaches two lines out, so this pins which values the ghosts take.
"""
import numpy as np
import pytest

from paper_1305_4736_amd import workloads as W


def test_uniform_state_is_fixed_point(orc):
    c = W.random_smooth(12, 10, seed=3, nsteps=20)
    p = c["params"]
    f0 = orc.init(p, 1.3, 0.11, -0.07, 0.9)
    f1 = orc.advance(p, f0, 20)
    assert np.abs(f1 - f0).max() <= 1e-14 * np.abs(f0).max() * 20


@pytest.mark.parametrize("axis", ["x", "y"])
def test_walls_hold_a_matching_uniform_state(orc, axis):
    # walls along `axis`... the fluid moves along them at their speed, at a
    # density other than the walls' nominal one (the wall density follows the
    # pressure of the fluid node next to it)
    P = W.bc("periodic")
    if axis == "y":
        w = W.bc("wall", 1.0, 0.1, 0.0, 0.9)
        bcs, state = [P, P, w, w], (1.3, 0.1, 0.0, 0.9)
    else:
        w = W.bc("wall", 1.0, 0.0, -0.08, 0.9)
        bcs, state = [w, w, P, P], (1.3, 0.0, -0.08, 0.9)
    c = W.random_smooth(12, 10, seed=4, bcs=bcs)
    p = c["params"]
    f0 = orc.init(p, *state)
    f1 = orc.advance(p, f0, 30)
    assert np.abs(f1 - f0).max() <= 1e-13 * np.abs(f0).max()
    # and a wall whose temperature differs from the fluid's does move it
    w2 = W.bc("wall", 1.0, w["state"][1], w["state"][2], 1.0)
    p2 = dict(p, bc=[w2 if b["kind"] == "wall" else b for b in p["bc"]])
    f2 = orc.advance(p2, orc.init(p2, *state), 30)
    assert np.abs(f2 - f0).max() > 1e-6 * np.abs(f0).max()


def _totals(orc, p, f):
    v, M, Mi, A = orc.constants(p["eta0"])
    m = np.einsum("ki,iyx->kyx", M[:4], f)
    return m.reshape(4, -1).sum(axis=1)


@pytest.mark.parametrize("limiter", ["mc", "minmod", "lw", "upwind"])
def test_conservation_periodic(orc, limiter):
    c = W.random_smooth(16, 12, seed=11, limiter=limiter, jumps=True)
    p = c["params"]
    f = orc.init(p, c["rho"], c["ux"], c["uy"], c["T"])
    t0 = _totals(orc, p, f)
    f = orc.advance(p, f, 60)
    t1 = _totals(orc, p, f)
    scale = np.array([abs(t0[0]), abs(t0[0]), abs(t0[0]), abs(t0[3])])
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale), (t0, t1)
    # the state did change (the test is not vacuous)
    assert np.abs(f - orc.init(p, c["rho"], c["ux"], c["uy"], c["T"])).max() > 1e-3


def _rot_field(a):
    """new[y', x'] = old[(-x') mod ny, y'] : the field rotated by +90 degrees
    (an ny x nx array becomes nx x ny)."""
    ny, nx = a.shape
    yp, xp = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    return a[(-xp) % ny, yp]


def test_rotation_symmetry(orc):
    n = 14
    c = W.random_smooth(n, n, seed=5, jumps=True, nsteps=25)
    p = c["params"]
    r, ux, uy, T = c["rho"], c["ux"], c["uy"], c["T"]
    fa = orc.run(p, r, ux, uy, T, 25)
    ra, uxa, uya, Ta = orc.macros(p, fa)
    # rotate the initial state: scalars move, velocity vectors turn by +90 degrees
    fb = orc.run(p, _rot_field(r), -_rot_field(uy), _rot_field(ux), _rot_field(T), 25)
    rb, uxb, uyb, Tb = orc.macros(p, fb)
    assert np.abs(rb - _rot_field(ra)).max() < 1e-12
    assert np.abs(Tb - _rot_field(Ta)).max() < 1e-12
    assert np.abs(uxb - (-_rot_field(uya))).max() < 1e-12
    assert np.abs(uyb - _rot_field(uxa)).max() < 1e-12


def test_rotation_symmetry_with_unequal_spacings(orc):
    # a rectangular grid with dy != dx: turning the state by 90 degrees swaps
    # the axes together with their spacings (a dx / dy mix-up in the velocity
    # gradients of the correction or in the Courant numbers breaks it)
    c = W.random_smooth(14, 10, seed=6, jumps=True, nsteps=25)
    p = dict(c["params"])
    dx = p["dx"]
    p.update(dy=1.6 * dx, dt=0.3 * dx / 6.0)
    pr = dict(p, nx=p["ny"], ny=p["nx"], dx=p["dy"], dy=p["dx"])
    r, ux, uy, T = c["rho"], c["ux"], c["uy"], c["T"]
    fa = orc.run(p, r, ux, uy, T, 25)
    ra, uxa, uya, Ta = orc.macros(p, fa)
    fb = orc.run(pr, _rot_field(r), -_rot_field(uy), _rot_field(ux), _rot_field(T), 25)
    rb, uxb, uyb, Tb = orc.macros(pr, fb)
    assert np.abs(ra - orc.macros(p, orc.run(p, r, ux, uy, T, 0))[0]).max() > 1e-6   # it moved
    assert np.abs(rb - _rot_field(ra)).max() < 1e-12
    assert np.abs(Tb - _rot_field(Ta)).max() < 1e-12
    assert np.abs(uxb - (-_rot_field(uya))).max() < 1e-12
    assert np.abs(uyb - _rot_field(uxa)).max() < 1e-12


def test_mirror_symmetry(orc):
    n = 12
    c = W.random_smooth(n, 9, seed=8, jumps=True, nsteps=25)
    p = c["params"]
    mir = lambda a: a[:, (-np.arange(n)) % n]
    fa = orc.run(p, c["rho"], c["ux"], c["uy"], c["T"], 25)
    ra, uxa, uya, Ta = orc.macros(p, fa)
    fb = orc.run(p, mir(c["rho"]), -mir(c["ux"]), mir(c["uy"]), mir(c["T"]), 25)
    rb, uxb, uyb, Tb = orc.macros(p, fb)
    assert np.abs(rb - mir(ra)).max() < 1e-12
    assert np.abs(uxb + mir(uxa)).max() < 1e-12
    assert np.abs(uyb - mir(uya)).max() < 1e-12
    assert np.abs(Tb - mir(Ta)).max() < 1e-12


def test_single_row_equals_uniform_rows(orc):
    c1 = W.sod(nx=80)
    c8 = W.sod(nx=80, ny=8)
    n = 150
    f1 = orc.run(c1["params"], c1["rho"], c1["ux"], c1["uy"], c1["T"], n)
    f8 = orc.run(c8["params"], c8["rho"], c8["ux"], c8["uy"], c8["T"], n)
    for y in range(8):
        assert np.abs(f8[:, y, :] - f1[:, 0, :]).max() < 1e-13


def test_boundaries_do_not_act_ahead_of_waves(orc):
    """Equilibrium / outflow / periodic x-boundaries only differ near the edge:
    after n steps the stencil (reach 2 nodes per step) has carried the
    difference at most 2n nodes inward."""
    c = W.riemann_1d((1.0, 0.2, 1.0), (0.5, 0.2, 0.6), 1.4, 120, nsteps=0)
    n = 20
    outs = []
    for kinds in (("equilibrium", "equilibrium"), ("outflow", "outflow"), ("periodic", "periodic")):
        p = dict(c["params"])
        p["bc"] = [dict(c["params"]["bc"][0], kind=kinds[0]), dict(c["params"]["bc"][1], kind=kinds[1]),
                   c["params"]["bc"][2], c["params"]["bc"][3]]
        outs.append(orc.run(p, c["rho"], c["ux"], c["uy"], c["T"], n))
    inner = slice(2 * n + 1, 120 - 2 * n - 1)
    for o in outs[1:]:
        assert np.abs(o[:, :, inner] - outs[0][:, :, inner]).max() == 0.0
    # and the periodic wrap does differ near the edges
    assert np.abs(outs[2] - outs[0]).max() > 1e-8


@pytest.mark.parametrize("kind", ["outflow", "equilibrium"])
@pytest.mark.parametrize("axis", ["x", "y"])
def test_ghosts_act_as_the_lines_they_stand_for(orc, kind, axis):
    E = W.bc("equilibrium", 1.1, 0.05, -0.02, 0.9)
    P, O = W.bc("periodic"), W.bc("outflow")
    bcs = [P, P, P, P]
    lo, hi = (0, 1) if axis == "x" else (2, 3)
    bcs[lo], bcs[hi] = O, (O if kind == "outflow" else E)
    nx, ny = 20, 14
    c = W.random_smooth(nx, ny, seed=8, bcs=bcs, jumps=True)
    p = c["params"]
    f = orc.init(p, c["rho"], c["ux"], c["uy"], c["T"])
    g = orc.advance(p, f, 1)
    # the same state on a grid four lines longer past the side under test
    ax = 2 if axis == "x" else 1                 # f is (plane, y, x)
    if kind == "outflow":
        last = np.take(f, [-1], axis=ax)
        extra = np.repeat(last, 4, axis=ax)
    else:
        line = dict(p, nx=4 if axis == "x" else nx, ny=ny if axis == "x" else 4,
                    bc=[P, P, P, P])
        extra = orc.init(line, *E["state"])
    fe = np.concatenate([f, extra], axis=ax)
    pe = dict(p, nx=nx + 4 if axis == "x" else nx, ny=ny + 4 if axis == "y" else ny)
    ge = orc.advance(pe, fe, 1)
    ge = ge[:, :, :nx] if axis == "x" else ge[:, :ny, :]
    assert np.abs(ge - g).max() <= 1e-13 * np.abs(g).max()
