"""Accuracy of every workload against the FP64 oracle, as a table.

    python tests/accuracy_report.py [--json PATH]   (needs the GPU and the built library)

Runs each configuration on the GPU through the C ABI and the same inputs
through the serial FP64 oracle, and prints the relative L1 and Linf errors
of rho, u_x, u_y and T (definitions in tests/parity.py) next to the bar
(1e-11 for FP64 storage, 2e-5 for FP32 storage).  Grids the oracle cannot
run in full within seconds are checked on windows (the full shock-interface
grid) or on a subset (the batch); the step counts are stated.  This is test
infrastructure like the parity tests, which assert the same bars; this
script only reports the figures.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from parity import TOL, rel_errors, window_params  # noqa: E402
from paper_1305_4736_amd import workloads as W  # noqa: E402

ROWS = []


def gamma_of(p):
    return (p["b"] + 2.0) / p["b"]


def record(name, precision, steps, per_launch, gpu, orc, gamma):
    e = rel_errors(gpu, orc, gamma)
    worst = max(max(v) for v in e.values())
    ROWS.append({"workload": name, "precision": precision, "steps": steps, "steps_per_launch": per_launch,
                 "errors": {k: [float(a), float(b)] for k, (a, b) in e.items()}, "worst": float(worst),
                 "bar": TOL[precision], "ok": bool(worst <= TOL[precision])})
    print(f"[accuracy] {name} {precision}: worst {worst:.2e} (bar {TOL[precision]:.0e})", flush=True)


def solve(mrtfd, case, n, per_launch=None):
    with mrtfd.Solver(case["params"]) as s:
        if per_launch:
            s.steps_per_launch = per_launch
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(n)
        s.sync()
        return s.macros(), s.steps_per_launch


def oracle_macros(case, n, p=None):
    p = p or case["params"]
    p64 = dict(p, precision="fp64")
    f = oracle.run(p64, case["rho"], case["ux"], case["uy"], case["T"], n)
    return oracle.macros(p64, f)


def whole(mrtfd, name, case, n, per_launch=None):
    mg, k = solve(mrtfd, case, n, per_launch)
    record(name, case["params"]["precision"], n, k, mg, oracle_macros(case, n), gamma_of(case["params"]))


def shock_interface_windows(mrtfd, precision, n=20):
    case = W.shock_interface(precision=precision)
    ny, nx = case["rho"].shape
    mg, k = solve(mrtfd, case, n)
    margin = 2 * n + 2
    gs, os_ = [[] for _ in range(4)], [[] for _ in range(4)]
    for x0, y0 in [(0, 100), (880, 0), (940, 250), (1000, 700), (nx - 128, 500), (960, ny - 64)]:
        nxw, nyw = 128, 128
        sl = lambda a: np.take(np.take(a, range(y0, y0 + nyw), axis=0, mode="wrap"), range(x0, x0 + nxw), axis=1)
        p = window_params(case["params"], x0, nxw, y0, nyw, keep_x_lo=(x0 == 0), keep_x_hi=(x0 + nxw == nx))
        sub = {"rho": sl(case["rho"]), "ux": sl(case["ux"]), "uy": sl(case["uy"]), "T": sl(case["T"])}
        mo = oracle_macros(sub, n, p)
        xs = slice(0 if x0 == 0 else margin, nxw if x0 + nxw == nx else nxw - margin)
        ys = slice(margin, nyw - margin)
        for q in range(4):
            gs[q].append(sl(mg[q])[ys, xs].ravel())
            os_[q].append(mo[q][ys, xs].ravel())
    record(f"shock_interface 4096x1024, 6 windows of 128x128 (interiors {128 - 2 * margin}x{128 - 2 * margin})",
           precision, n, k, [np.concatenate(g) for g in gs], [np.concatenate(o) for o in os_], 1.4)


def batch_subset(mrtfd, n=100):
    cases, _ = W.riemann_batch(n=512, precision="fp32")
    small = sorted((c for c in cases if c["params"]["nx"] * c["params"]["ny"] <= 20000),
                   key=lambda c: c["params"]["nx"] * c["params"]["ny"])
    cases = [small[round(i * (len(small) - 1) / 15)] for i in range(16)]
    with mrtfd.Batch(len(cases), precision="fp32") as b:
        slots = [b.add(c["params"], c["rho"], c["ux"], c["uy"], c["T"]) for c in cases]
        b.autotune()
        b.step(n)
        b.status()
        gpu = [b.macros(s) for s in slots]
    gs, os_ = [[] for _ in range(4)], [[] for _ in range(4)]
    worst = None
    for c, mg in zip(cases, gpu):
        mo = oracle_macros(c, n)
        e = rel_errors(mg, mo, gamma_of(c["params"]))
        w = max(max(v) for v in e.values())
        worst = w if worst is None else max(worst, w)
        for q in range(4):
            gs[q].append(np.ravel(mg[q]))
            os_[q].append(np.ravel(mo[q]))
    # errors pooled over the 16 instances (each instance also within the bar)
    record("riemann batch: 16 of the 512 instances (up to 20000 nodes), one batch", "fp32", n, 1,
           [np.concatenate(g) for g in gs], [np.concatenate(o) for o in os_], 1.4)
    ROWS[-1]["worst_single_instance"] = float(worst)


def served(mrtfd, serve):
    rng = np.random.default_rng(5)
    reqs, t = [], 0.0
    for k in range(14):
        t += rng.exponential(0.002)
        spec = W.serve_request(rng, k, log_lo=8, log_hi=48)
        spec["nsteps"] = int(rng.integers(5, 60))
        reqs.append((t, spec))
    with serve.Server(capacity=3, steps_per_tick=7, keep_results=True, reserve_bytes=0) as srv:
        rep = srv.run(reqs, realtime=True)
    for prec in ("fp64", "fp32"):
        gs, os_ = [[] for _ in range(4)], [[] for _ in range(4)]
        for i, (_, spec) in enumerate(reqs):
            case = W.spec_case(spec)
            if case["params"]["precision"] != prec:
                continue
            mo = oracle_macros(case, spec["nsteps"])
            for q in range(4):
                gs[q].append(np.ravel(rep["results"][i][q]))
                os_[q].append(np.ravel(mo[q]))
        record(f"served stream: the {prec} requests of 14 (quadrants and Couette, 8..48 per side)", prec,
               "5..59", 1, [np.concatenate(g) for g in gs], [np.concatenate(o) for o in os_], 1.4)


# ----------------------------------------------------------------------------
# FP32 storage against FP64 storage, both on the GPU, at the configured
# lengths the oracle cannot reach in seconds (the FP64 path itself is within
# 5e-14 of the oracle on every case above).

FP32_ROWS = []


def record32(name, steps, gpu32, gpu64, gamma, extra=None):
    e = rel_errors(gpu32, gpu64, gamma)
    row = {"workload": name, "steps": steps, "errors": {k: [float(a), float(b)] for k, (a, b) in e.items()},
           "worst": float(max(max(v) for v in e.values()))}
    row.update(extra or {})
    FP32_ROWS.append(row)
    print(f"[accuracy-fp32] {name}: worst {row['worst']:.2e}", flush=True)


def fp32_vs_fp64_shock_interface(mrtfd, n=2000):
    out = {}
    for prec in ("fp32", "fp64"):
        out[prec], _ = solve(mrtfd, W.shock_interface(precision=prec), n)
    record32("shock_interface 4096x1024, full grid", n, out["fp32"], out["fp64"], 1.4)


def fp32_vs_fp64_batch(mrtfd, n=1000):
    res = {}
    for prec in ("fp32", "fp64"):
        cases, _ = W.riemann_batch(n=512, precision=prec)
        with mrtfd.Batch(len(cases), precision=prec) as b:
            slots = [b.add(c["params"], c["rho"], c["ux"], c["uy"], c["T"]) for c in cases]
            b.autotune()
            b.step(n)
            b.status()
            res[prec] = [b.macros(s) for s in slots]
    worst = []
    for c, g32, g64 in zip(cases, res["fp32"], res["fp64"]):
        e = rel_errors(g32, g64, gamma_of(c["params"]))
        worst.append((max(v[1] for v in e.values()), max(v[0] for v in e.values())))
    linf = sorted(w[0] for w in worst)
    pooled32 = [np.concatenate([np.ravel(g[q]) for g in res["fp32"]]) for q in range(4)]
    pooled64 = [np.concatenate([np.ravel(g[q]) for g in res["fp64"]]) for q in range(4)]
    record32("riemann batch, all 512 instances (pooled; per instance below)", n, pooled32, pooled64, 1.4,
             {"per_instance_linf_median": float(linf[len(linf) // 2]), "per_instance_linf_max": float(linf[-1]),
              "per_instance_l1_max": float(max(w[1] for w in worst)),
              "instances_linf_over_2e-5": int(sum(1 for v in linf if v > 2e-5))})


def fp32_vs_fp64_served(mrtfd, count=24):
    reqs = W.serve_stream(seed=13054737, max_requests=count)
    worst = []
    for _, spec in reqs:
        case = W.spec_case(spec)
        out = {}
        for prec in ("fp32", "fp64"):
            c = dict(case, params=dict(case["params"], precision=prec))
            out[prec], _ = solve(mrtfd, c, spec["nsteps"])
        e = rel_errors(out["fp32"], out["fp64"], gamma_of(case["params"]))
        worst.append((spec["kind"], spec["params"]["nx"], spec["params"]["ny"], spec["nsteps"],
                      max(v[1] for v in e.values()), max(v[0] for v in e.values())))
    for kind in ("quadrant", "couette"):
        w = [x for x in worst if x[0] == kind]
        if not w:
            continue
        FP32_ROWS.append({"workload": f"served requests ({kind}), the first {count} of the stream, each alone",
                          "steps": "200..5000", "count": len(w),
                          "linf_max": float(max(x[4] for x in w)), "l1_max": float(max(x[5] for x in w)),
                          "linf_over_2e-5": int(sum(1 for x in w if x[4] > 2e-5)),
                          "cases": [list(x[1:]) for x in w]})
        print(f"[accuracy-fp32] served {kind}: {len(w)} requests, Linf max {max(x[4] for x in w):.2e}, "
              f"L1 max {max(x[5] for x in w):.2e}", flush=True)


def fp32_vs_fp64_couette(mrtfd, n=20000):
    for pr in (0.5, 1.0, 2.0):
        out = {}
        for prec in ("fp32", "fp64"):
            c = W.couette(pr=pr)
            c["params"]["precision"] = prec
            out[prec], _ = solve(mrtfd, c, n)
        record32(f"thermal Couette 4x200, Pr = {pr}", n, out["fp32"], out["fp64"], 1.4)


def main():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    from paper_1305_4736_amd import mrtfd, serve
    import test_gpu_paper_runs as paper

    oracle._load()
    for prec in ("fp64", "fp32"):
        whole(mrtfd, "Sod 400x1, minmod, full run to t = 0.15", W.sod(precision=prec), 3600)
    for prec in ("fp64", "fp32"):
        c = W.couette(pr=1.0)
        c["params"]["precision"] = prec
        whole(mrtfd, "thermal Couette 4x200, Pr = 1, gamma = 1.4 (walls)", c, 20000)
    for prec in ("fp64", "fp32"):
        shock_interface_windows(mrtfd, prec)
    for prec in ("fp64", "fp32"):
        c = W.random_smooth(300, 200, seed=3, bcs=[W.bc("equilibrium", 1.1, 0.05, -0.02, 0.9), W.bc("outflow"),
                                                  W.bc("periodic"), W.bc("periodic")],
                            precision=prec, jumps=True)
        whole(mrtfd, "random smooth 300x200 with jumps, two steps per launch forced", c, 40, per_launch=2)
    batch_subset(mrtfd)
    served(mrtfd, serve)
    whole(mrtfd, "Sec. IV-A discontinuity 1000x1, MC, to t = 0.06", paper.discontinuity("mc"), 6000)
    c, *_ = paper.lax_tube(500)
    whole(mrtfd, "Sec. IV-B Lax tube 1000x1 (first 500 steps)", c, 500)
    whole(mrtfd, "Sec. V heavy/light 1200x10 (first 1000 steps)", W.paper_heavy_light(), 1000)

    print("\n| workload | storage | steps | steps per launch | rho L1 / Linf | u_x L1 / Linf | u_y L1 / Linf "
          "| T L1 / Linf | bar |")
    print("|---|---|---|---|---|---|---|---|---|")
    for r in ROWS:
        e = r["errors"]
        cell = lambda k: f"{e[k][0]:.1e} / {e[k][1]:.1e}"
        print(f"| {r['workload']} | {r['precision']} | {r['steps']} | {r['steps_per_launch']} | {cell('rho')} | "
              f"{cell('ux')} | {cell('uy')} | {cell('T')} | {r['bar']:.0e}{'' if r['ok'] else ' EXCEEDED'} |")

    fp32_vs_fp64_shock_interface(mrtfd)
    fp32_vs_fp64_batch(mrtfd)
    fp32_vs_fp64_served(mrtfd)
    fp32_vs_fp64_couette(mrtfd)
    print("\nFP32 storage against FP64 storage (both on the GPU):\n")
    for r in FP32_ROWS:
        print(json.dumps(r))
    if "--json" in sys.argv:
        with open(sys.argv[sys.argv.index("--json") + 1], "w") as fh:
            json.dump({"against_oracle": ROWS, "fp32_against_fp64": FP32_ROWS}, fh, indent=1)


if __name__ == "__main__":
    main()
