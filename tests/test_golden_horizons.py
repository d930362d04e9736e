"""The stored oracle results of the long-horizon parity tests
(tests/golden/make_oracle_horizons.py) against what they must satisfy.

* couette_steady_oracle.json: one case re-run with the oracle gives the same
  profiles; every case meets the steady-state criterion it was stopped by, u
  is the analytic linear profile and the viscous-heating bump of T grows
  with Pr (Sec. IV-C; the analytic bump is Pr u_0^2 / (8 c_p) at mid-channel).
* shock_interface_window_oracle.json: the sampled nodes behind the incoming
  shock hold the inflow state the run started from (a uniform equilibrium
  region does not move), and the sample reaches into the waves.
"""
import json
import os

import numpy as np

from paper_1305_4736_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_couette_golden_properties():
    cases = load("couette_steady_oracle.json")["cases"]
    assert [c["pr"] for c in cases] == [0.5, 1.0, 2.0]
    bumps = []
    for c in cases:
        assert c["steps"] % 5000 == 0 and c["last_step_change"] < 1e-10
        y = np.arange(200) / 199.0
        ua, Ta = W.couette_analytic(y, c["pr"], c["gamma"])
        assert np.abs(np.asarray(c["ux"]) - ua).max() < 2e-4 * 0.2
        assert np.abs(np.asarray(c["uy"])).max() < 1e-5
        bump = np.asarray(c["T"])[100] - 1.0
        assert abs(bump / (Ta[100] - 1.0) - 1.0) < 0.2
        bumps.append(bump)
    assert 3.0 < bumps[2] / bumps[0] < 4.6


def test_couette_golden_is_the_oracle_run(orc):
    c = load("couette_steady_oracle.json")["cases"][2]
    case = W.couette(pr=c["pr"], gamma=c["gamma"], nx=1)
    p = case["params"]
    f = orc.run(p, case["rho"], case["ux"], case["uy"], case["T"], c["steps"])
    m = orc.macros(p, f)
    for k, q in enumerate(("rho", "ux", "uy", "T")):
        assert np.array_equal(m[k][:, 0], np.asarray(c[q])), q


def test_shock_window_golden_properties():
    g = load("shock_interface_window_oracle.json")
    x, y = np.asarray(g["x"]), np.asarray(g["y"])
    assert g["steps"] == 200 and g["oracle_columns"] - x.max() - 1 >= 2 * g["steps"] + 2
    r2, u2, p2, _ = W.normal_shock(5.0, 1.0, 2.0, 1.4)
    behind = x < 900
    assert behind.sum() > 100
    rho, ux, T = (np.asarray(g[q]) for q in ("rho", "ux", "T"))
    assert np.abs(rho[behind] - r2).max() < 1e-12 * r2
    assert np.abs(ux[behind] - u2).max() < 1e-12
    assert np.abs(T[behind] - p2 / r2).max() < 1e-12
    # the waves: light gas (rho ~ 1), heavy gas (rho ~ 5) and the shocked states
    assert rho.min() < 1.5 and ((rho > 4.0) & (rho < 6.0)).any() and rho.max() > 13.0
