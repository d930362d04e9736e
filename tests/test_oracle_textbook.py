"""Special cases of the flux-limiter convection that reduce to textbook
schemes for linear advection (Sec. III, limiter discussion).

With every relaxation rate zero and the energy-flux correction off, the
collision vanishes and each f_i is advected on its own along x.  Then

* at Courant number 1 (dt = dx / 6 for the |v| = 6 axis group) the update is
  an exact one-cell shift;
* psi = 0 is first-order upwind, psi = 1 is Lax-Wendroff;
* the MC and minmod limiters give the textbook flux-limited Lax-Wendroff
  scheme (LeVeque's form with phi(r) applied to the upwind jump ratio) and are
  total-variation diminishing.

The textbook schemes are written below in their own standard notation, as
whole-array numpy updates, not with the oracle's node-by-node formulas.
"""
import numpy as np
import pytest

from paper_1305_4736_amd import workloads as W

NX = 24


def _free_streaming_case(limiter, dt, dy_over_dx=1.0):
    d = 1.0 / NX
    s = [0.0] * 16
    p = W.make_params(NX, 1, d, dy_over_dx * d, dt, s, 5.0, [W.bc("periodic")] * 4, limiter=limiter,
                      correction=False)
    return p


def _random_f(orc, p, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(NX) / NX
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x + 0.3)[None, :]
    ux = 0.2 * np.cos(4 * np.pi * x)[None, :]
    T = 1.0 + 0.2 * np.sin(6 * np.pi * x)[None, :]
    f = orc.init(p, rho, ux, 0.0, T)
    f = f + 0.05 * rng.standard_normal(f.shape) * np.abs(f).mean()
    # a sharp step too, so the limiters have something to limit
    f[:, :, NX // 2:] += 0.1
    return f


def _vx(orc):
    v, M, Mi, A = orc.constants()
    return v[0]


def textbook_step(q, nu, phi):
    """One step of q_t + c q_x = 0 (c > 0, Courant nu) with the flux-limited
    Lax-Wendroff scheme: q_j - nu (q_j - q_{j-1})
    - nu (1 - nu)/2 [phi(r_j) (q_{j+1} - q_j) - phi(r_{j-1}) (q_j - q_{j-1})],
    r_j = (q_j - q_{j-1}) / (q_{j+1} - q_j), periodic."""
    qm, qp = np.roll(q, 1), np.roll(q, -1)
    dplus = qp - q
    dminus = q - qm
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(dplus != 0, dminus / np.where(dplus != 0, dplus, 1.0), 0.0)
    lim = np.where(dplus != 0, phi(r) * dplus, 0.0)
    return q - nu * dminus - 0.5 * nu * (1.0 - nu) * (lim - np.roll(lim, 1))


PHI = {
    "upwind": lambda r: np.zeros_like(r),
    "lw": lambda r: np.ones_like(r),
    "minmod": lambda r: np.maximum(0.0, np.minimum(1.0, r)),
    "mc": lambda r: np.maximum(0.0, np.minimum(np.minimum(2.0 * r, 0.5 * (1.0 + r)), 2.0)),
}


@pytest.mark.parametrize("limiter", ["upwind", "lw", "minmod", "mc"])
def test_reduces_to_textbook_limited_scheme(orc, limiter):
    dt = 0.4 * (1.0 / NX) / 6.0
    p = _free_streaming_case(limiter, dt)
    f0 = _random_f(orc, p, 1)
    f1 = orc.advance(p, f0, 1)
    vx = _vx(orc)
    for i in range(16):
        c = vx[i]
        if c == 0.0:
            # no x-component; y is periodic with one row, so nothing moves
            assert np.abs(f1[i] - f0[i]).max() < 1e-15
            continue
        nu = abs(c) * dt * NX
        q = f0[i, 0] if c > 0 else f0[i, 0, ::-1]
        ref = textbook_step(q, nu, PHI[limiter])
        if c < 0:
            ref = ref[::-1]
        assert np.abs(f1[i, 0] - ref).max() < 1e-14 * (1 + np.abs(q).max()), (limiter, i)


def test_unit_courant_is_exact_shift(orc, dy_over_dx=1.0):
    dt = (1.0 / NX) / 6.0
    for limiter in ("mc", "minmod", "lw", "upwind"):
        p = _free_streaming_case(limiter, dt, dy_over_dx)
        f0 = _random_f(orc, p, 2)
        f1 = orc.advance(p, f0, 1)
        vx = _vx(orc)
        for i in range(16):
            if abs(abs(vx[i]) - 6.0) < 1e-12:
                shift = 1 if vx[i] > 0 else -1
                ref = np.roll(f0[i], shift, axis=1)
                assert np.abs(f1[i] - ref).max() <= 4e-16 * np.abs(f0[i]).max() * 4


def test_unit_courant_is_exact_shift_with_unequal_spacings(orc):
    # the shift along x depends on dx alone (the one-row y axis is inert)
    test_unit_courant_is_exact_shift(orc, dy_over_dx=2.0)


@pytest.mark.parametrize("limiter", ["minmod", "mc"])
def test_total_variation_diminishing(orc, limiter):
    dt = 0.9 * (1.0 / NX) / 6.0
    p = _free_streaming_case(limiter, dt)
    f = _random_f(orc, p, 3)
    tv = lambda a: np.abs(np.diff(np.concatenate([a, a[:1]]))).sum()
    vx = _vx(orc)
    tv0 = [tv(f[i, 0]) for i in range(16)]
    f = orc.advance(p, f, 30)
    for i in range(16):
        if vx[i] != 0.0:
            assert tv(f[i, 0]) <= tv0[i] * (1 + 1e-13)
    # Lax-Wendroff is not TVD on the same data (so the test can tell them apart)
    p_lw = _free_streaming_case("lw", dt)
    g = orc.advance(p_lw, _random_f(orc, p_lw, 3), 30)
    assert any(tv(g[i, 0]) > tv0[i] * 1.01 for i in range(16) if vx[i] != 0.0)
