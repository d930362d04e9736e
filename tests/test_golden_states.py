"""The paper's printed gas states (tests/golden/paper_states.json) pin the
workload recipes: the discontinuity test and the heavy/light run state that
their two sides satisfy the Hugoniot relations with gamma = 2 and a Mach 1.414
shock (Sec. IV-A, Sec. V); the Lax states satisfy p = rho T with R = 1."""
import json
import math
import os

import numpy as np

from paper_1305_4736_amd import workloads as W

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_states.json")))


def _rh_residuals(pre, post, gamma):
    """Jump conditions across a shock moving at speed S into `pre` (u = 0)."""
    r1, u1, p1 = pre
    r2, u2, p2 = post
    S = r2 * u2 / (r2 - r1)                          # mass
    E = lambda r, u, p: p / (gamma - 1) + 0.5 * r * u * u
    mom = r2 * u2 * (u2 - S) + p2 - p1               # momentum (u1 = 0)
    en = (E(r2, u2, p2) + p2) * u2 - S * (E(r2, u2, p2) - E(r1, u1, p1))
    return S, mom, en


def test_discontinuity_states_are_hugoniot():
    d = G["discontinuity_test"]
    L, R = d["left"], d["right"]
    S, mom, en = _rh_residuals((R["rho"], 0.0, R["rho"] * R["T"]),
                               (L["rho"], L["u1"], L["rho"] * L["T"]), d["gamma"])
    assert abs(S - 2.0) < 1e-4
    assert abs(mom) < 1e-4 and abs(en) < 1e-4


def test_heavy_light_states_and_recipe():
    h = G["heavy_light"]
    s, hv = h["shock"], h["heavy"]
    S, mom, en = _rh_residuals((hv["rho"], 0.0, hv["p"]), (s["rho"], s["u1"], s["p"]), h["gamma"])
    mach = S / math.sqrt(h["gamma"] * hv["p"] / hv["rho"])
    assert abs(mach - h["mach"]) < 1e-3
    assert abs(mom) < 1e-4 and abs(en) < 1e-4
    # the recipe uses the exact states (3/2, 2/3, 7/3) these print to 6 digits
    c = W.paper_heavy_light()
    p = c["params"]
    assert (p["nx"], p["ny"]) == tuple(h["cells"])
    assert abs(c["rho"][0, 0] - s["rho"]) < 1e-12
    assert abs(c["ux"][0, 0] - s["u1"]) < 1e-6
    assert abs(c["rho"][0, 0] * c["T"][0, 0] - s["p"]) < 1e-5
    assert abs(c["rho"][0, -1] - h["light"]["rho"]) < 1e-12
    assert abs(c["nsteps"] * p["dt"] - h["t_end"]) < 1e-12
    assert abs(p["b"] - 2.0) < 1e-12                 # gamma = 2


def test_recipe_rankine_hugoniot():
    r2, u2, p2, W_ = W.normal_shock(5.0, 1.0, 2.0, 1.4)
    S, mom, en = _rh_residuals((5.0, 0.0, 1.0), (r2, u2, p2), 1.4)
    assert abs(S - W_) < 1e-12 and abs(mom) < 1e-12 and abs(en) < 1e-12
    assert abs(r2 - 40.0 / 3.0) < 1e-12 and abs(p2 - 4.5) < 1e-12


def test_lax_states_pressure():
    lx = G["lax_tube"]
    for side, p_ref in (("left", 3.528), ("right", 0.571)):
        st = lx[side]
        assert abs(st["rho"] * st["T"] - p_ref) < 2e-3


def test_couette_prandtl_pairs():
    for gamma, pr, s5, s8 in G["couette_prandtl"]["pairs"]:
        assert abs(s8 / s5 - pr) < 1e-12
