"""The screen of the batched Riemann workload against the stored oracle
census of its draws (tests/golden/riemann_screen_envelope.json, written by
tests/golden/make_screen_envelope.py, which calls only the oracle).

* Under the workload's screen (temperature ratio 5, pressure ratio 7,
  subsonic) none of the 512 draws has a node with rho <= 0, T <= 0 or a
  non-finite value after any of its 1000 steps, and the census saw the
  same redraw count the builder reports.
* Every screen in the census that contains it and is wider has a failing
  draw, so it is the widest of those tried; the survey's temperature-ratio
  screen alone fails 58 of 512.
* Re-run with the oracle here: the smallest failing draw under the
  temperature-ratio screen does fail, and the smallest draws of the
  workload's screen stay finite.
"""
import json
import math
import os

import numpy as np

from paper_1305_4736_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def census():
    with open(os.path.join(GOLDEN, "riemann_screen_envelope.json")) as fh:
        return json.load(fh)


def bounds(entry):
    return tuple(math.inf if b is None else b for b in entry["bounds"])


def test_workload_screen_is_the_widest_finite_one():
    screens = census()["screens"]
    mine = [v for v in screens.values() if bounds(v) == W.SCREEN]
    assert len(mine) == 1
    assert mine[0]["nonfinite"] == 0
    _, redraws = W.riemann_batch(n=512, precision="fp64")
    assert mine[0]["redraws"] == redraws
    wider = [v for v in screens.values()
             if all(a >= b for a, b in zip(bounds(v), W.SCREEN)) and bounds(v) != W.SCREEN]
    assert len(wider) >= 8
    assert all(v["nonfinite"] >= 1 for v in wider)
    assert screens["t20"]["nonfinite"] == 58


def _run(orc, case, steps=1000):
    """Whether the draw keeps every node finite with rho > 0 and T > 0 after
    each of its steps (the census's criterion)."""
    p = dict(case["params"], ny=1, precision="fp64")
    rows = [np.ascontiguousarray(case[q][:1]) for q in ("rho", "ux", "uy", "T")]
    try:
        f = orc.init(p, *rows)
        for _ in range(steps):
            f = orc.advance(p, f, 1)
            r, _, _, T = orc.macros(p, f)
            if not (np.all(np.isfinite(f)) and r.min() > 0 and T.min() > 0):
                return False
    except ValueError:
        return False
    return True


def test_census_entries_rerun_with_the_oracle(orc):
    screens = census()["screens"]
    cases, _ = W.riemann_batch(n=512, precision="fp64", screen=bounds(screens["t20"]))
    bad = screens["t20"]["nonfinite_instances"]
    k = min(bad, key=lambda i: cases[i]["params"]["nx"])
    assert not _run(orc, cases[k])
    cases, _ = W.riemann_batch(n=512, precision="fp64")
    for k in sorted(range(512), key=lambda i: cases[i]["params"]["nx"])[:2]:
        assert _run(orc, cases[k]), k
