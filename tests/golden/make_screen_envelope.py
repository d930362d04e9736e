"""Count, with the oracle, how many of the 512 seeded Riemann draws of the
batched workload go non-finite, or reach rho <= 0 or T <= 0 at some node,
after any of their 1000 steps (the check the GPU path makes after every
step), under several screens of the drawn states.

    python tests/golden/make_screen_envelope.py [processes]

Writes tests/golden/riemann_screen_envelope.json (screens already in it are
kept, the others computed).  Only the oracle (oracle/)
and the seeded input builder (paper_1305_4736_amd.workloads) are used.  The
instances are uniform in y, so each runs as one row (the same run).  A
screen is (temperature ratio, pressure ratio, Mach number) bounds: draws
beyond them are redrawn from the same stream.
"""
from __future__ import annotations

import json
import math
import multiprocessing
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
STEPS = 1000
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

SCREENS = {
    "t20": (20.0, math.inf, math.inf),              # the survey's screen: temperature ratio 1/20
    "t20_subsonic": (20.0, math.inf, 1.0),
    "t10_p10_subsonic": (10.0, 10.0, 1.0),
    "t5_p5": (5.0, 5.0, math.inf),
    "t5_p5_subsonic": (5.0, 5.0, 1.0),             # the workload's screen
    "t7_p7_subsonic": (7.0, 7.0, 1.0),
    "t10_p5_subsonic": (10.0, 5.0, 1.0),
    "t5_p10_subsonic": (5.0, 10.0, 1.0),
    "t5_p20_subsonic": (5.0, 20.0, 1.0),
    "t5_subsonic": (5.0, math.inf, 1.0),
    "t6_p10_subsonic": (6.0, 10.0, 1.0),
    "t6_p20_subsonic": (6.0, 20.0, 1.0),
    "t7_p10_subsonic": (7.0, 10.0, 1.0),
    "t5_p7_subsonic": (5.0, 7.0, 1.0),
    "t6_p6_subsonic": (6.0, 6.0, 1.0),
    "t6_p7_subsonic": (6.0, 7.0, 1.0),
}


def run_one(args):
    """(k, first failing step or None): a draw fails at the first step after
    which some node holds a non-finite population, rho <= 0 or T <= 0 (the
    check the GPU path makes after every step)."""
    import oracle
    k, p, rows = args
    try:
        f = oracle.init(p, *rows)
        for s in range(STEPS):
            f = oracle.advance(p, f, 1)
            r, _, _, T = oracle.macros(p, f)
            if not (np.all(np.isfinite(f)) and r.min() > 0 and T.min() > 0):
                return k, s + 1
    except ValueError:
        return k, 0
    return k, None


def main(procs):
    from paper_1305_4736_amd import workloads as W
    path = os.path.join(HERE, "riemann_screen_envelope.json")
    out = {"source": "tests/golden/make_screen_envelope.py (oracle only)", "steps": STEPS,
           "criterion": "non-finite, rho <= 0 or T <= 0 at any node after any step", "screens": {}}
    if os.path.exists(path):
        with open(path) as fh:
            out["screens"].update(json.load(fh).get("screens", {}))
    for name, scr in SCREENS.items():
        if name in out["screens"]:
            continue
        t0 = time.time()
        cases, redraws = W.riemann_batch(n=512, precision="fp64", screen=scr)
        work, ratios = [], []
        for k, c in enumerate(cases):
            p = dict(c["params"], ny=1)
            work.append((k, p, [np.ascontiguousarray(c[q][:1]) for q in ("rho", "ux", "uy", "T")]))
            bl, br = p["bc"][0]["state"], p["bc"][1]["state"]
            ratios.append({"T_ratio": max(bl[3], br[3]) / min(bl[3], br[3]),
                           "p_ratio": max(bl[0] * bl[3], br[0] * br[3]) / min(bl[0] * bl[3], br[0] * br[3])})
        del cases
        with multiprocessing.Pool(procs) as pool:
            res = pool.map(run_one, work, chunksize=4)
        fail = {k: s for k, s in res if s is not None}
        bad = sorted(fail)
        out["screens"][name] = {"bounds": [b if math.isfinite(b) else None for b in scr], "redraws": redraws,
                                "nonfinite": len(bad), "nonfinite_instances": bad,
                                "first_failing_step": [fail[k] for k in bad],
                                "nonfinite_states": [ratios[k] for k in bad]}
        print(f"{name}: {redraws} redraws, {len(bad)} of 512 non-finite ({time.time() - t0:.0f} s)", flush=True)
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 6)
