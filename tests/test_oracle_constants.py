"""Pins of the oracle's constants and equilibria against what the paper fixes.

* the velocity set (Sec. II, Fig. 1) as a set of 16 vectors, and A_i (Sec. III);
* M M^-1 = I (the inverse is a true inverse of the Appendix matrix);
* the seven moment relations (Appendix, relations a-g) satisfied by
  f^eq = M^-1 fhat^eq, which pins the rows of M, the inverse and every one of
  the twelve non-conserved equilibria at once (a dropped term, a sign or a
  swapped row breaks at least one relation).
"""
import itertools
import math

import numpy as np
import pytest


def paper_velocities():
    r2 = math.sqrt(2.0)
    vs = []
    for mag in (1.0, 6.0):
        vs += [(mag, 0.0), (-mag, 0.0), (0.0, mag), (0.0, -mag)]
    for c in (r2, 3.0 / r2):
        vs += [(sx * c, sy * c) for sx in (1, -1) for sy in (1, -1)]
    return np.array(vs)


def test_velocity_set_matches_paper(orc):
    v, M, Mi, A = orc.constants()
    mine = sorted(map(tuple, np.round(v.T, 12)))
    ref = sorted(map(tuple, np.round(paper_velocities(), 12)))
    assert mine == ref
    speeds = np.hypot(v[0], v[1])
    assert np.allclose(sorted(set(np.round(speeds, 12))), [1.0, 2.0, 3.0, 6.0])
    # A_i |v_ia| is 0 or 1 for every component (Sec. III)
    prod = np.abs(A[None, :] * v)
    assert np.all((np.abs(prod) < 1e-15) | (np.abs(prod - 1.0) < 1e-14))


def test_inverse(orc):
    v, M, Mi, A = orc.constants()
    I = np.eye(16)
    assert np.abs(M @ Mi - I).max() < 1e-13
    assert np.abs(Mi @ M - I).max() < 1e-13
    # no accidental singularity: conditioning of the 16x16 basis
    assert np.linalg.cond(M) < 1e4
    assert abs(np.linalg.det(M)) > 1e20


def test_first_rows_are_conserved_moments(orc):
    """Rows 1..4 are 1, v_x, v_y, v^2 + eta^2 (Appendix m_1..m_4) with eta = 5/2
    on the |v| = 1 group only (Appendix, after the relations)."""
    v, M, Mi, A = orc.constants()
    speeds = np.hypot(v[0], v[1])
    eta = np.where(np.abs(speeds - 1.0) < 1e-12, 2.5, 0.0)
    assert np.allclose(M[0], 1.0)
    assert np.allclose(M[1], v[0])
    assert np.allclose(M[2], v[1])
    assert np.allclose(M[3], speeds ** 2 + eta ** 2)


def _relations(f, vx, vy, eta, rho, ux, uy, T, b):
    """Residuals of the seven moment relations (Appendix a-g), R = 1."""
    P = rho * T
    u = (ux, uy)
    v = (vx, vy)
    u2 = ux * ux + uy * uy
    vv = vx * vx + vy * vy + eta * eta
    res = []
    res.append(np.sum(f) - rho)                                                 # (a)
    for a in range(2):
        res.append(np.sum(f * v[a]) - rho * u[a])                               # (b)
    res.append(np.sum(f * vv) - rho * (b * T + u2))                             # (c)
    for a, bb in itertools.product(range(2), repeat=2):
        res.append(np.sum(f * v[a] * v[bb]) - (P * (a == bb) + rho * u[a] * u[bb]))   # (d)
    for a in range(2):
        res.append(np.sum(f * vv * v[a]) - rho * ((b + 2) * T + u2) * u[a])     # (e)
    for a, bb, c in itertools.product(range(2), repeat=3):
        rhs = rho * (T * (u[a] * (bb == c) + u[bb] * (a == c) + u[c] * (a == bb))
                     + u[a] * u[bb] * u[c])
        res.append(np.sum(f * v[a] * v[bb] * v[c]) - rhs)                       # (f)
    for a, bb in itertools.product(range(2), repeat=2):
        d = float(a == bb)
        rhs = rho * ((b + 2) * T * T * d + ((b + 4) * u[a] * u[bb] + u2 * d) * T
                     + u2 * u[a] * u[bb])
        res.append(np.sum(f * vv * v[a] * v[bb]) - rhs)                         # (g)
    return np.array(res)


@pytest.mark.parametrize("b", [2.0, 3.0, 5.0, 2.0 / 0.67])
def test_seven_moment_relations(orc, b):
    rng = np.random.default_rng(int(b * 1000))
    v, M, Mi, A = orc.constants()
    speeds = np.hypot(v[0], v[1])
    eta = np.where(np.abs(speeds - 1.0) < 1e-12, 2.5, 0.0)
    for _ in range(25):
        rho = rng.uniform(0.1, 10.0)
        ux, uy = rng.uniform(-0.8, 0.8, 2)
        T = rng.uniform(0.05, 3.0)
        f = orc.feq(rho, ux, uy, T, b)
        res = _relations(f, v[0], v[1], eta, rho, ux, uy, T, b)
        scale = rho * (1.0 + T + ux * ux + uy * uy) ** 2
        assert np.abs(res).max() / scale < 1e-13, res


def test_feq_hat_consistent_with_velocity_space(orc):
    """M f^eq reproduces fhat^eq (the Appendix closed forms) for the conserved
    inputs rho, j, e (Sec. II: e = b rho T + rho u^2)."""
    v, M, Mi, A = orc.constants()
    rng = np.random.default_rng(7)
    for _ in range(10):
        rho, T, b = rng.uniform(0.2, 5), rng.uniform(0.1, 2), rng.uniform(1.5, 8)
        ux, uy = rng.uniform(-0.5, 0.5, 2)
        e = rho * (b * T + ux * ux + uy * uy)
        fh = orc.feq_hat(rho, rho * ux, rho * uy, e, b)
        f = orc.feq(rho, ux, uy, T, b)
        assert np.allclose(M @ f, fh, rtol=1e-13, atol=1e-13 * np.abs(fh).max())


def test_eta_enters_only_through_m(orc):
    """eta changes M (rows with v^2 + eta^2) but the equilibrium moments of
    the seven relations do not depend on it."""
    v, M1, _, _ = orc.constants(2.5)
    _, M2, _, _ = orc.constants(1.5)
    diff_rows = np.where(np.abs(M1 - M2).max(axis=1) > 0)[0]
    assert set(diff_rows) == {3, 7, 8, 13, 15}   # row 15 vanishes on the eta group
    f1 = orc.feq(1.2, 0.1, -0.2, 0.8, 5.0, eta0=2.5)
    f2 = orc.feq(1.2, 0.1, -0.2, 0.8, 5.0, eta0=1.5)
    # same density, momentum and pressure tensor
    for w in (np.ones(16), v[0], v[1], v[0] * v[0], v[0] * v[1], v[1] * v[1]):
        assert abs(np.dot(w, f1) - np.dot(w, f2)) < 1e-13
