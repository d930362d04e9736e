#!/usr/bin/env python3
"""Benchmark of the fused D2V16 MRT-FD step on one MI355X.

Workload: the heavy/light shock-interface problem on a 4096 x 1024 grid
(Mach-2 shock in rho = 5 gas, sinusoidal interface to rho = 1 gas, inflow /
outflow in x, periodic in y, MC limiter), FP64 storage, with the Delta*
fields computed every 100 steps.  A "step" is one explicit stage of the
whole grid; value = interior node-updates per second over the timed steps,
inputs resident in HBM.

Printed: ONE JSON line with the contract fields plus
  roofline     -- the step kernel's algorithmic HBM bytes per launch
                  (16 reads + 16 writes of f per node-update; an FP64 launch
                  takes two steps, i.e. two node-updates per node) over its
                  average launch time, measured with HIP events on the
                  library's stream inside the timed region; traffic (the HBM
                  bytes the launch actually moves) from the committed
                  rocprofv3 counter summary when it matches the current kernel
  cpu_baseline -- the FP64 oracle on the host, on a bounded sample of the
                  same workload (a few full-grid steps)
  fp64_one_step_per_launch -- the FP64 workload with one step per launch
                  (the default takes two)
  fp32_storage -- the same workload with f stored and convected in FP32
                  (and fp32_one_step_per_launch)
  limiters_fp64_ms_per_step -- the FP64 step time with each limiter (MC,
                  minmod, Lax-Wendroff, first-order upwind)
  small_configs_fp64_us_per_step -- the latency-bound 400 x 1 Sod tube and
                  4 x 200 thermal Couette flow, device microseconds per step
  batched      -- 512 independent Riemann instances of uneven size in one
                  batch (FP32 storage, autotuned shape classes)
  served       -- a Poisson stream of solve requests (Riemann quadrants and
                  thermal Couette flows, 64..2048 per side, 200..5000 steps,
                  FP32 / FP64) served with continuous batching: p50 / p99
                  latency, offered and achieved node-updates/s; at the
                  specified 200 requests/s (overloaded), at the highest rate
                  measured to keep a bounded queue (25 requests/s, drained)
                  and at a light 15 requests/s (drained).

Options --pmc-copy-calibration, --no-cpu-baseline, --no-limiters,
--no-batched, --no-serve and --steps-per-launch serve the profiling runs
(see profiles/).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "node-updates/s (D2V16 MRT-FD) + % HBM peak; p50/p99 served-solve latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_march2_shock_interface_4096x1024.json")


def code_tokens(text: str, line_comment: str) -> str:
    """The text without comments and with whitespace runs collapsed (string
    literals kept whole), so that editing a comment does not change a hash."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith(line_comment, i):
            while i < n and text[i] != "\n":
                i += 1
        elif line_comment == "//" and text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif c.isspace():
            while i < n and text[i].isspace():
                i += 1
            if out and out[-1] != " ":
                out.append(" ")
        else:
            out.append(c)
            i += 1
    return "".join(out).strip()


def kernel_hash() -> str:
    """Hash of the code that builds and launches the single-instance step
    kernels (the sources other than the batched entry points, and the build
    flags; comments and whitespace aside): the stored traffic counters are
    reported only while it matches."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_1305_4736_amd")
    csrc = os.path.join(pkg, "csrc")
    files = [os.path.join(csrc, n) for n in sorted(os.listdir(csrc)) if n != "mrtfd_batch.hip"]
    for path in files + [os.path.join(pkg, "build.py")]:
        with open(path, encoding="utf-8") as fh:
            text = fh.read()
        h.update(os.path.basename(path).encode())
        h.update(code_tokens(text, "#" if path.endswith(".py") else "//").encode())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_node(precision: str) -> int:
    return 32 * (8 if precision == "fp64" else 4)


def run_gpu(case, steps, warmup, noneq_every, log, per_launch=0):
    import torch

    from paper_1305_4736_amd import mrtfd

    p = case["params"]
    nx, ny = p["nx"], p["ny"]
    dev = torch.device("cuda:0")
    fields = [torch.tensor(case[k], dtype=torch.float64, device=dev) for k in ("rho", "ux", "uy", "T")]
    delta = torch.empty((16, ny, nx), dtype=torch.float64, device=dev) if noneq_every else None
    s = mrtfd.Solver(p, stream=torch.cuda.current_stream())
    if per_launch:
        s.steps_per_launch = per_launch
    s.init(*fields)
    del fields
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    log(f"[bench] {case['name']} {p['precision']}: warm-up {warmup} steps done")

    kernel_ms = 0.0
    done = 0
    t0 = time.perf_counter()
    while done < steps:
        chunk = min(noneq_every or steps, steps - done)
        kernel_ms += s.step_timed(chunk)
        done += chunk
        if noneq_every and done % noneq_every == 0:
            s.noneq(star=True, out=delta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.sync()
    elapsed = t1 - t0
    nodes = nx * ny
    res = {
        "elapsed_s": elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "value": nodes * steps / elapsed,
        "kernel_ms_avg": kernel_ms / steps,
        "nodes": nodes,
        "steps_per_launch": s.steps_per_launch,
    }
    s.close()
    del delta
    torch.cuda.empty_cache()
    log(f"[bench] {case['name']} {p['precision']}: {steps} steps in {elapsed:.3f} s, "
        f"{res['value']:.4e} node-updates/s, kernel {res['kernel_ms_avg']:.4f} ms")
    return res


def roofline(res, precision):
    # the step timer brackets whole chunks of launches; with two steps per
    # launch (even chunks) a launch lasts two step-times and processes two
    # node-updates per node
    k = res["steps_per_launch"]
    bytes_launch = algorithmic_bytes_per_node(precision) * res["nodes"] * k
    launch_ms = res["kernel_ms_avg"] * k
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    kernel = "k_march2" if k == 2 else "k_march"
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        if t.get("kernel_hash") == kernel_hash() and t.get("precision") == precision and t.get("kernel") == kernel:
            traffic = t["hbm_bytes_per_launch"]
    out = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "algorithmic_bytes_per_launch": bytes_launch, "kernel": kernel, "steps_per_launch": k,
           "avg_launch_ms": round(launch_ms, 5)}
    if k == 2:
        out["note"] = ("two steps per launch: achieved counts 256 B per node-update, two per node; the launch "
                       "moves about half that (traffic) and is bound by FP64 VALU issue")
    return out


def cpu_baseline(log, nsteps=6):
    """The FP64 oracle (serial C) on `nsteps` steps of the full grid."""
    import oracle
    from paper_1305_4736_amd import workloads as W

    case = W.shock_interface()
    p = case["params"]
    f = oracle.init(p, case["rho"], case["ux"], case["uy"], case["T"])
    t0 = time.perf_counter()
    oracle.advance(p, f, nsteps)
    dt = time.perf_counter() - t0
    nodes = p["nx"] * p["ny"]
    log(f"[bench] cpu oracle: {nsteps} full-grid steps in {dt:.1f} s")
    return {"value": nodes * nsteps / dt, "unit": "node-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{nsteps} steps of the full {p['nx']}x{p['ny']} grid, serial FP64 C oracle "
                      f"(gcc -O2), {dt:.1f} s"}


def run_limiters(log, steps=100):
    """Step time with each limiter (the same workload, FP64, the library's
    default steps per launch): MC, minmod, Lax-Wendroff (psi = 1),
    first-order upwind (psi = 0)."""
    import torch

    from paper_1305_4736_amd import mrtfd, workloads as W

    out = {}
    for lim in ("mc", "minmod", "lw", "upwind"):
        case = W.shock_interface(precision="fp64", limiter=lim)
        s = mrtfd.Solver(case["params"], stream=torch.cuda.current_stream())
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(10)
        out[lim] = s.step_timed(steps) / steps
        s.sync()
        s.close()
    log("[bench] limiters (fp64 ms/step): " + ", ".join(f"{k} {v:.4f}" for k, v in out.items()))
    return out


def run_small(log, steps=2000):
    """Latency-bound small configurations, as device microseconds per step
    (FP64): the 400 x 1 Sod tube and the 4 x 200 thermal Couette flow."""
    import torch

    from paper_1305_4736_amd import mrtfd, workloads as W

    out = {}
    for name, case in (("sod_400x1", W.sod()), ("couette_4x200_pr1", W.couette(pr=1.0))):
        s = mrtfd.Solver(case["params"], stream=torch.cuda.current_stream())
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(100)
        out[name] = 1e3 * s.step_timed(steps) / steps
        s.sync()
        s.close()
    log("[bench] small configs (fp64 us/step): " + ", ".join(f"{k} {v:.2f}" for k, v in out.items()))
    return out


def run_batched(steps, warmup, log, n=512):
    """512 independent Riemann instances (log-uniform Nx in [128, 4096], Ny in
    [1, 256], seeded states) in one batch, FP32 storage, autotuned shape
    classes."""
    from paper_1305_4736_amd import mrtfd, workloads as W

    cases, redraws = W.riemann_batch(n=n, precision="fp32")
    nodes = sum(c["params"]["nx"] * c["params"]["ny"] for c in cases)
    b = mrtfd.Batch(n, precision="fp32", limiter="mc")
    for c in cases:
        b.add(c["params"], c["rho"], c["ux"], c["uy"], c["T"])
    costs = b.autotune()
    names = list(mrtfd.SHAPE_CLASSES)
    shapes = {}
    for k in range(n):
        tx, ty = b.shape(k)
        sh = "strips" if tx == 60 else f"tile{tx}x{ty}"
        shapes[sh] = shapes.get(sh, 0) + 1
    b.step(warmup)
    b.sync()
    ms = b.step_timed(steps)
    try:
        b.status()
        nonfinite = 0
    except mrtfd.NonFiniteError as e:
        nonfinite = int((e.flags != 0).sum())
    b.close()
    value = nodes * steps / (ms * 1e-3)
    log(f"[bench] batched {n} instances, {nodes} nodes: {ms / steps:.4f} ms/step, {value:.4e} node-updates/s")
    return {"workload": f"riemann_batch_{n}", "instances": n, "nodes": nodes, "precision": "fp32",
            "limiter": "mc", "steps": steps, "ms_per_step": ms / steps, "value": value,
            "unit": "node-updates/s", "screen_redraws": redraws, "nonfinite_instances": nonfinite,
            "autotune_us_per_unit": dict(zip(names, map(float, costs))),
            "shape_classes": shapes}


def run_served(rate, seconds, log, drain, label, steps_per_tick=50, capacity=4096, cap_bytes=None):
    """Poisson stream of MRT-FD solve requests served with continuous batching."""
    from paper_1305_4736_amd import serve, workloads as W

    reqs = W.serve_stream(rate=rate, duration=seconds)
    with serve.Server(capacity=capacity, steps_per_tick=steps_per_tick, max_resident_bytes=cap_bytes) as srv:
        rep = srv.run(reqs, duration=seconds, drain=drain, log=log)
    rep = {k: v for k, v in rep.items() if k != "results"}
    rep.update({"label": label, "rate_per_s": rate, "arrival_window_s": seconds, "drained": drain})
    log(f"[bench] served ({label}): {rep['completed']}/{rep['requests']} done, p50 {rep['p50_s']:.3f} s, "
        f"p99 {rep['p99_s']:.3f} s, achieved {rep['achieved_node_updates_per_s']:.3e} node-updates/s")
    return rep


def copy_calibration(log, nbytes=1 << 30):
    """A plain device copy of known size, for scaling rocprofv3 byte counters."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: 3 copies of {nbytes} bytes")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--noneq-every", type=int, default=100)
    ap.add_argument("--steps-per-launch", type=int, default=0, choices=(0, 1, 2),
                    help="force one or two steps per kernel launch (0: the library's default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--pmc-copy-calibration", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-limiters", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=8.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    # the highest of 20, 25, 30 and 35 requests/s whose queue stayed bounded
    # (at 30 the offered load exceeds what the device achieves)
    ap.add_argument("--sustainable-rate", type=float, default=25.0)
    ap.add_argument("--light-rate", type=float, default=15.0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "a multi-GPU run (slabs along y with one halo exchange per step) is designed but not built.", file=sys.stderr)
        sys.exit(2)

    log = lambda m: print(m, file=sys.stderr, flush=True)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    from paper_1305_4736_amd import workloads as W

    if args.pmc_copy_calibration:
        copy_calibration(log)

    case = W.shock_interface(precision="fp64")
    res = run_gpu(case, args.steps, args.warmup, args.noneq_every, log, args.steps_per_launch)
    rl = roofline(res, "fp64")

    extra = {}
    if not args.steps_per_launch and res["steps_per_launch"] == 2:
        # the same workload with one step per launch, for comparison
        r1 = run_gpu(case, args.steps, args.warmup, args.noneq_every, log, 1)
        rl1 = roofline(r1, "fp64")
        extra["fp64_one_step_per_launch"] = {"value": r1["value"], "ms_per_step": r1["ms_per_step"],
                                             "kernel_ms_per_step": round(r1["kernel_ms_avg"], 5),
                                             "roofline_frac": rl1["frac"], "achieved_GBs": rl1["achieved"]}
    if not args.no_fp32:
        case32 = W.shock_interface(precision="fp32")
        r32 = run_gpu(case32, args.steps, args.warmup, args.noneq_every, log, args.steps_per_launch)
        rl32 = roofline(r32, "fp32")
        extra["fp32_storage"] = {"value": r32["value"], "ms_per_step": r32["ms_per_step"],
                                 "steps_per_launch": r32["steps_per_launch"],
                                 "roofline_frac": rl32["frac"], "achieved_GBs": rl32["achieved"],
                                 "speedup_vs_fp64": r32["value"] / res["value"]}
        if not args.steps_per_launch and r32["steps_per_launch"] == 2:
            r1 = run_gpu(case32, args.steps, args.warmup, args.noneq_every, log, 1)
            extra["fp32_one_step_per_launch"] = {"value": r1["value"], "ms_per_step": r1["ms_per_step"],
                                                 "kernel_ms_per_step": round(r1["kernel_ms_avg"], 5),
                                                 "roofline_frac": roofline(r1, "fp32")["frac"]}

    if not args.no_limiters:
        extra["limiters_fp64_ms_per_step"] = run_limiters(log)
        extra["small_configs_fp64_us_per_step"] = run_small(log)

    if not args.no_batched:
        extra["batched"] = run_batched(max(args.steps // 2, 20), 5, log)
    if not args.no_serve:
        extra["served"] = run_served(args.serve_rate, args.serve_seconds, log, drain=False,
                                     label="offered load as specified (overloaded), stopped at the end of arrivals")
        extra["served_sustainable"] = run_served(args.sustainable_rate, args.serve_seconds, log, drain=True,
                                                 label="highest sustainable rate measured, drained")
        extra["served_light"] = run_served(args.light_rate, args.serve_seconds, log, drain=True,
                                           label="light load, drained")

    cpu = None if args.no_cpu_baseline else cpu_baseline(log)

    line = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "shock_interface_4096x1024", "grid": [4096, 1024], "precision": "fp64",
                   "limiter": "mc", "noneq_star_every": args.noneq_every, "gamma": 1.4,
                   "boundaries": "inflow / outflow in x, periodic in y"},
        "roofline": rl,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
