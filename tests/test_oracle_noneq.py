"""Pins of the non-equilibrium diagnostics (Sec. V, Appendix M*).

Delta = M (f - f^eq) and Delta* = M*(u) (f - f^eq), M* being M with v
replaced by v - u.  What the mathematics fixes:

* at equilibrium both vanish;
* Delta_1..4 = Delta*_1..4 = 0 for any f (f and f^eq share rho, j, e);
* where u = 0, Delta* = Delta;
* because the first four components vanish, the second-order central moments
  equal the raw ones: Delta*_5..7 = Delta_5..7 for any u;
* for the third-order ones the binomial shift gives, e.g.,
  Delta*_10 = Delta_10 - 3 u_x Delta_5' ... written here in terms of the raw
  second-order moments Pxx, Pxy, Pyy of (f - f^eq).

The profile values of the paper's Fig. 6 are not printed, so the numbers
themselves are "parity unpinned"; these identities are what is checked.
"""
import numpy as np

from paper_1305_4736_amd import workloads as W


def _state(orc, seed=4, nsteps=30):
    c = W.random_smooth(10, 8, seed=seed, jumps=True)
    p = c["params"]
    f = orc.run(p, c["rho"], c["ux"], c["uy"], c["T"], nsteps)
    return p, f


def test_zero_at_equilibrium(orc):
    c = W.random_smooth(6, 5, seed=2)
    p = c["params"]
    f = orc.init(p, c["rho"], c["ux"], c["uy"], c["T"])
    for star in (False, True):
        d = orc.noneq(p, f, star)
        assert np.abs(d).max() < 1e-12


def test_conserved_components_vanish(orc):
    p, f = _state(orc)
    for star in (False, True):
        d = orc.noneq(p, f, star)
        scale = np.abs(d).max()
        assert scale > 1e-6
        assert np.abs(d[:4]).max() < 1e-12 * max(1.0, scale) * 100


def test_star_equals_plain_at_rest(orc):
    c = W.random_smooth(8, 6, seed=9)
    p = c["params"]
    f = orc.init(p, c["rho"], 0.0, 0.0, c["T"])
    # perturb, then remove the momentum the perturbation added, node by node
    v, M, Mi, A = orc.constants()
    rng = np.random.default_rng(1)
    f = f + 1e-3 * rng.standard_normal(f.shape)
    j = np.einsum("ki,iyx->kyx", M[1:3], f)
    rho = np.einsum("i,iyx->yx", M[0], f)
    # f <- f - rho^-1 * (j . v) * w with w a fixed velocity-space vector of unit mass
    w = np.zeros(16)
    w[0] = w[2] = 0.5   # (1,0) and (-1,0): zero net momentum, unit mass
    wx = np.zeros(16)
    wx[0], wx[2] = 0.5, -0.5   # unit x-momentum, zero mass
    wy = np.zeros(16)
    wy[1], wy[3] = 0.5, -0.5
    f = f - j[0][None] * wx[:, None, None] - j[1][None] * wy[:, None, None]
    r, ux, uy, T = orc.macros(p, f)
    assert np.abs(ux).max() < 1e-14 and np.abs(uy).max() < 1e-14
    d = orc.noneq(p, f, False)
    ds = orc.noneq(p, f, True)
    assert np.abs(d - ds).max() < 1e-13 * np.abs(d).max()


def test_central_moment_shift_identities(orc):
    p, f = _state(orc, seed=6)
    v, M, Mi, A = orc.constants()
    r, ux, uy, T = orc.macros(p, f)
    d = orc.noneq(p, f, False)
    ds = orc.noneq(p, f, True)
    scale = np.abs(d).max()
    # second order: identical
    for k in (4, 5, 6):
        assert np.abs(ds[k] - d[k]).max() < 1e-12 * scale
    # third order, translational part: sum c_x (c_x^2 + c_y^2) g with c = v - u and
    # sum g = sum v g = 0 gives Delta*_10 = Delta_10 - 2 (ux Pxx + uy Pxy) - ux (Pxx + Pyy)
    Pxx = 0.5 * (d[4] + d[5])
    Pyy = 0.5 * (d[4] - d[5])
    Pxy = d[6]
    ref10 = d[9] - 2 * (ux * Pxx + uy * Pxy) - ux * (Pxx + Pyy)
    ref11 = d[10] - 2 * (ux * Pxy + uy * Pyy) - uy * (Pxx + Pyy)
    assert np.abs(ds[9] - ref10).max() < 1e-11 * scale
    assert np.abs(ds[10] - ref11).max() < 1e-11 * scale
