#!/usr/bin/env python3
"""Benchmark of the fused D2V16 MRT-FD step on one MI355X.

Workload: the heavy/light shock-interface problem on a 4096 x 1024 grid
(Mach-2 shock in rho = 5 gas, sinusoidal interface to rho = 1 gas, inflow /
outflow in x, periodic in y, MC limiter), FP64 storage, with the Delta*
fields computed every 100 steps.  A "step" is one explicit stage of the
whole grid; value = interior node-updates per second over the timed steps,
inputs resident in HBM.

Printed: ONE JSON line with the contract fields plus
  roofline     -- the step kernel against the nearer of two roofs: VALU
                  issue (SQ_INSTS_VALU per launch) and HBM (the bytes the
                  launch moves, FETCH_SIZE + WRITE_SIZE scaled by kernels of
                  known traffic), both from the committed rocprofv3 counter
                  summary when it matches the current kernel code, over the
                  average launch time measured with HIP events on the
                  library's stream inside the timed region; beside them the
                  algorithmic rate (16 reads + 16 writes of f per
                  node-update; a two-step launch counts two node-updates per
                  node) as hbm_effective
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
import math
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
    """State bytes read and written per node-update: 16 populations in FP64
    (2 x 128 B), or in FP32 storage 16 FP32 populations and 4 FP64
    conserved moments (2 x 96 B)."""
    return 256 if precision == "fp64" else 192


def run_gpu(case, steps, warmup, noneq_every, log, per_launch=0, keep_macros=False):
    """The workload's timed steps.  The Delta* pass runs after every
    `noneq_every` steps inside the timed region and is charged at that rate
    into `value`: with fewer timed steps than that (the short default runs),
    one pass is timed after the region and its time times steps / noneq_every
    is added to the steps' wall time."""
    import torch

    from paper_1305_4736_amd import mrtfd

    p = case["params"]
    nx, ny = p["nx"], p["ny"]
    dev = torch.device("cuda:0")
    fields = [torch.tensor(case[k], dtype=torch.float64, device=dev) for k in ("rho", "ux", "uy", "T")]
    delta = torch.empty((16, ny, nx), dtype=torch.float64, device=dev) if noneq_every else None
    stream = torch.cuda.current_stream()
    s = mrtfd.Solver(p, stream=stream)
    if per_launch:
        s.steps_per_launch = per_launch
    s.init(*fields)
    del fields
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    log(f"[bench] {case['name']} {p['precision']}: warm-up {warmup} steps done")

    def noneq_timed():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.noneq(star=True, out=delta)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1)

    stamps = torch.zeros((2, 16), dtype=torch.int64, device=dev)
    kernel_ms = 0.0
    noneq_ms = []
    done = 0
    mrtfd.clock_stamp(stamps, 0, stream)
    t0 = time.perf_counter()
    while done < steps:
        chunk = min(noneq_every or steps, steps - done)
        kernel_ms += s.step_timed(chunk)
        done += chunk
        if noneq_every and done % noneq_every == 0:
            noneq_ms.append(noneq_timed())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mrtfd.clock_stamp(stamps, 1, stream)
    s.sync()
    inside = len(noneq_ms)
    if noneq_every and not noneq_ms:
        noneq_ms.append(noneq_timed())
    st = stamps.cpu().tolist()
    clock = mrtfd.clock_mhz(st)
    wall_steps = (t1 - t0) - 1e-3 * sum(noneq_ms[:inside])
    noneq_avg = (sum(noneq_ms) / len(noneq_ms)) if noneq_ms else 0.0
    charged = wall_steps + (steps / noneq_every if noneq_every else 0.0) * 1e-3 * noneq_avg
    nodes = nx * ny
    res = {
        "elapsed_s": charged,
        "ms_per_step": 1e3 * charged / steps,
        "value": nodes * steps / charged,
        "steps_wall_s": wall_steps,
        "kernel_ms_avg": kernel_ms / steps,
        "noneq_ms": noneq_avg,
        "noneq_passes_in_region": inside,
        "clock_mhz": clock,
        "nodes": nodes,
        "steps_per_launch": s.steps_per_launch,
    }
    if keep_macros:
        res["macros"] = s.macros()
    s.close()
    del delta
    torch.cuda.empty_cache()
    log(f"[bench] {case['name']} {p['precision']}: {steps} steps in {wall_steps:.4f} s (+ Delta* charged "
        f"{charged - wall_steps:.5f} s), {res['value']:.4e} node-updates/s, kernel {res['kernel_ms_avg']:.4f} ms "
        f"per step, clock estimate {clock:.0f} MHz")
    return res


# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per
# SIMD every 4 cycles (16 lanes per cycle: a wave64 FP64 FMA, or any other
# wave64 VALU instruction, takes 4 cycles); 6.144e11 wave64 instructions/s,
# which is the published 78.6 TFLOP/s FP64 vector peak when each lane does
# an FMA.
VALU_PEAK = 256 * 4 * 2.4e9 / 4


def roofline(res, precision):
    """The step kernel's place under its two roofs, from its live average
    launch time and the counters of the committed profile (when they were
    taken on the current kernel code): VALU issue (SQ_INSTS_VALU per
    dispatch) against the VALU peak, and HBM traffic (FETCH_SIZE +
    WRITE_SIZE) against 8 TB/s.  `bound` is the roof the kernel is closer to;
    `achieved`/`peak`/`frac` are that roof's.  The algorithmic HBM rate (256
    or 192 bytes per node-update, two node-updates per node with two steps
    per launch) is reported beside it as `hbm_effective`."""
    k = res["steps_per_launch"]
    bytes_launch = algorithmic_bytes_per_node(precision) * res["nodes"] * k
    launch_s = res["kernel_ms_avg"] * k * 1e-3
    kernel = "k_march2" if k == 2 else "k_march"
    eff = bytes_launch / launch_s / 1e9
    ctr = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        if t.get("kernel_hash") == kernel_hash():
            ctr = t.get("kernels", {}).get(f"{kernel}/{precision}")
    traffic = ctr["hbm_bytes_per_launch"] if ctr else None
    valu = ctr["valu_insts_per_launch"] if ctr else None
    hbm = None if traffic is None else traffic / launch_s / 1e9
    valu_rate = None if valu is None else valu / launch_s
    clock = res.get("clock_mhz")
    out = {"traffic": traffic, "kernel": kernel, "steps_per_launch": k, "avg_launch_ms": round(launch_s * 1e3, 5),
           "hbm_effective": {"algorithmic_bytes_per_launch": bytes_launch, "GBs": round(eff, 2),
                             "frac": round(eff / HBM_PEAK_GBS, 4)},
           "hbm_measured": None if hbm is None else {"GBs": round(hbm, 2), "frac": round(hbm / HBM_PEAK_GBS, 4)},
           "valu": None if valu is None else {
               "insts_per_launch": valu, "per_s": valu_rate, "frac": round(valu_rate / VALU_PEAK, 4)},
           # shader-clock counter over real-time counter around the timed
           # region, mean over the XCDs: follows the clock within a run, but
           # has read above the 2.4 GHz maximum on some machines, so no
           # figure is derived from it
           "core_clock_mhz_estimate": round(clock, 1) if clock else None}
    if valu is not None and hbm is not None and valu_rate / VALU_PEAK >= hbm / HBM_PEAK_GBS:
        out.update({"bound": "alu", "achieved": valu_rate, "peak": VALU_PEAK, "unit": "VALU instr/s (wave64)",
                    "frac": round(valu_rate / VALU_PEAK, 4)})
    elif hbm is not None:
        out.update({"bound": "hbm", "achieved": round(hbm, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm / HBM_PEAK_GBS, 4)})
    else:
        # no counters for this code: the algorithmic rate is all there is
        out.update({"bound": "hbm", "achieved": round(eff, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(eff / HBM_PEAK_GBS, 4), "note": "no counter profile of this kernel code: "
                    "achieved is the algorithmic (effective) rate"})
    return out


def macro_errors(a, b, gamma):
    """Relative L1 / Linf errors of (rho, ux, uy, T) a against b: rho and T
    over their own sums / maxima, velocities over the flow speed's (the
    sound speed only for a flow slower than 1e-3 of it)."""
    import numpy as np
    speed = np.hypot(b[1], b[2])
    cs = math.sqrt(gamma * float(np.abs(b[3]).max()))
    slow = speed.max() < 1e-3 * cs
    den_u = (cs * speed.size, cs) if slow else (float(speed.sum()), float(speed.max()))
    out = {}
    for k, name in enumerate(("rho", "ux", "uy", "T")):
        d = np.abs(np.asarray(a[k]) - np.asarray(b[k]))
        den = den_u if k in (1, 2) else (float(np.abs(b[k]).sum()), float(np.abs(b[k]).max()))
        out[name] = [float(d.sum() / den[0]), float(d.max() / den[1])]
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(log, nsteps=6):
    """The FP64 oracle (serial C, one thread) on `nsteps` steps of the full grid."""
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
                      f"(gcc -O2), {dt:.1f} s",
            "host_nproc": os.cpu_count(), "cpu_model": cpu_model()}


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
    pair_rows = b.pair_rows()
    b.close()
    value = nodes * steps / (ms * 1e-3)
    log(f"[bench] batched {n} instances, {nodes} nodes: {ms / steps:.4f} ms/step, {value:.4e} node-updates/s")
    return {"workload": f"riemann_batch_{n}", "instances": n, "nodes": nodes, "precision": "fp32",
            "limiter": "mc", "steps": steps, "ms_per_step": ms / steps, "value": value,
            "unit": "node-updates/s",
            "screen": {"T_ratio_max": W.SCREEN[0], "p_ratio_max": W.SCREEN[1], "mach_max": W.SCREEN[2]},
            "screen_redraws": redraws, "nonfinite_instances": nonfinite,
            "autotune_us_per_unit": dict(zip(names, map(float, costs))),
            "shape_classes": shapes, "pair_band_rows": pair_rows}


def run_served(rate, seconds, log, drain, label, steps_per_tick=50, capacity=4096, cap_bytes=None,
               policy="fifo", latency_target_s=2.0, shed_after_s=4.0):
    """Poisson stream of MRT-FD solve requests served with continuous
    batching, admitted first come first served by memory (policy "fifo") or
    with the resident work bounded by a latency target, smallest work first,
    shedding what could not start within shed_after_s (policy "latency")."""
    from paper_1305_4736_amd import serve, workloads as W

    reqs = W.serve_stream(rate=rate, duration=seconds)
    with serve.Server(capacity=capacity, steps_per_tick=steps_per_tick, max_resident_bytes=cap_bytes,
                      policy=policy, latency_target_s=latency_target_s, shed_after_s=shed_after_s) as srv:
        rep = srv.run(reqs, duration=seconds, drain=drain, log=log)
    rep = {k: v for k, v in rep.items() if k != "results"}
    rep.update({"label": label, "rate_per_s": rate, "arrival_window_s": seconds, "drained": drain})
    log(f"[bench] served ({label}): {rep['completed']}/{rep['requests']} done, {rep['shed']} shed, "
        f"{rep['failed']} failed, p50 {rep['p50_s']:.3f} s, p99 {rep['p99_s']:.3f} s (completed only), "
        f"achieved {rep['achieved_node_updates_per_s']:.3e} node-updates/s")
    return rep


PROFILE_KERNELS = {"k_march2/fp64": "k_march2<0, double>", "k_march/fp64": "k_march<0, double>",
                   "k_march2/fp32": "k_march2<0, float>", "k_march/fp32": "k_march<0, float>",
                   "k_march2_batch/fp32": "k_march2_batch<0, float>", "k_march_batch/fp32": "k_march_batch<0, float>"}
PROFILE_COMMAND = ("python3 bench.py --steps 20 --warmup 4 --no-cpu-baseline --no-limiters "
                   "--no-serve --pmc-copy-calibration")


def _counter_rows(d):
    """(kernel name, counter name, value) of every dispatch in a rocprofv3
    --pmc CSV output directory."""
    import csv
    import glob
    out = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                out.append((r["Dispatch_Id"], r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    return out


def summarize_profile(fetch_dir, write_dir, sq_dir, out_path):
    """Per-launch HBM bytes and VALU instructions of the step kernels from
    three rocprofv3 --pmc runs of PROFILE_COMMAND (FETCH_SIZE; WRITE_SIZE;
    SQ_INSTS_VALU, SQ_WAVES, GRBM_GUI_ACTIVE), the byte counters scaled by
    what they read for kernels of known traffic in the same run: WRITE_SIZE
    by a plain 1 GiB device copy's writes, FETCH_SIZE by the FP64
    initialisation of the same grid, which reads 32 B per node in the step
    kernels' access pattern (8-byte loads per lane, whole lines).  (The
    copy's reads, in wider loads, read differently on the same counter;
    its factor is kept as a cross-check.)"""
    def per_kernel(rows, counter):
        acc = {}
        for disp, name, cname, val in rows:
            if cname != counter:
                continue
            acc.setdefault(name, {}).setdefault(disp, 0.0)
            acc[name][disp] += val
        return acc

    fetch = per_kernel(_counter_rows(fetch_dir), "FETCH_SIZE")
    write = per_kernel(_counter_rows(write_dir), "WRITE_SIZE")
    sq_rows = _counter_rows(sq_dir)
    valu = per_kernel(sq_rows, "SQ_INSTS_VALU")
    waves = per_kernel(sq_rows, "SQ_WAVES")
    gui = per_kernel(sq_rows, "GRBM_GUI_ACTIVE")
    gib = float(1 << 30)
    # the calibration copies: the dispatches that write 1 GiB, and the same
    # dispatches (same program, same launch order) in the fetch pass
    cal = {(name, disp) for name, d in write.items() for disp, v in d.items() if abs(v * 1024 - gib) < 0.01 * gib}
    cw = [write[name][disp] for name, disp in cal]
    cf = [fetch[name][disp] for name, disp in cal if disp in fetch.get(name, {})]
    if not cw or len(cf) != len(cw):
        raise RuntimeError("calibration copies not found in both passes")
    copy_fetch_factor = gib / (1024 * sum(cf) / len(cf))
    write_factor = gib / (1024 * sum(cw) / len(cw))

    def match(d, inst):
        vals = [v for name, dd in d.items() if inst in name for v in dd.values()]
        return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)

    nodes = 4096 * 1024
    # the FP64 initialisation of the 4096 x 1024 grid: four FP64 fields
    # read (32 B per node), 16 FP64 populations written (128 B per node)
    fi, ni = match(fetch, "k_init<double>")
    wi, _ = match(write, "k_init<double>")
    if fi is None or wi is None:
        raise RuntimeError("the FP64 initialisation kernel is missing from the counter passes")
    fetch_factor = 32 * nodes / (1024 * fi)
    kernels = {}
    for key, inst in PROFILE_KERNELS.items():
        kname, prec = key.split("/")
        f, nf = match(fetch, inst)
        w, nw = match(write, inst)
        v, nv = match(valu, inst)
        wv, _ = match(waves, inst)
        g, _ = match(gui, inst)
        if f is None or w is None:
            continue
        fb, wb = 1024 * f * fetch_factor, 1024 * w * write_factor
        k = 2 if kname.startswith("k_march2") else 1
        # (the batched launches' node counts vary from launch to launch: no
        # algorithmic count per launch for them)
        alg = None if kname.endswith("_batch") else algorithmic_bytes_per_node(prec) * nodes * k
        kernels[key] = {"instance": inst, "dispatches": {"fetch": nf, "write": nw, "sq": nv},
                        "fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
                        "hbm_bytes_per_launch": round(fb + wb), "algorithmic_bytes_per_launch": alg,
                        "hbm_over_algorithmic": round((fb + wb) / alg, 4) if alg else None,
                        "valu_insts_per_launch": v, "waves_per_launch": wv, "valu_insts_per_wave": v / wv if wv else None,
                        "grbm_gui_active_per_launch": g}
    fetch_cal = {"kernel": "k_init<double>", "dispatches": ni, "read_bytes": 32 * nodes,
                 "fetch_factor": fetch_factor,
                 # its writes, scaled by the copy's write factor, against its 128 B per node
                 "write_over_expected": round(1024 * wi * write_factor / (128 * nodes), 4)}
    out = {"workload": "shock_interface_4096x1024 (single-grid kernels), riemann_batch_512 (batched)",
           "kernel_hash": kernel_hash(),
           "command": PROFILE_COMMAND, "passes": ["FETCH_SIZE", "WRITE_SIZE", "SQ_INSTS_VALU SQ_WAVES GRBM_GUI_ACTIVE"],
           "copy_calibration": {"bytes": int(gib), "fetch_factor": copy_fetch_factor, "write_factor": write_factor},
           "fetch_calibration": fetch_cal,
           "kernels": kernels}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def summarize_counters(dirs):
    """Mean per dispatch of every counter in rocprofv3 --pmc CSV output
    directories, for each step kernel of PROFILE_KERNELS (counters summed
    over a dispatch's rows), with the number of dispatches."""
    out = {}
    for d in dirs:
        per = {}
        for disp, name, cname, val in _counter_rows(d):
            inst = next((i for i in PROFILE_KERNELS.values() if i in name), None)
            if inst is None:
                continue
            per.setdefault(inst, {}).setdefault(cname, {}).setdefault(disp, 0.0)
            per[inst][cname][disp] += val
        for inst, cs in per.items():
            o = out.setdefault(inst, {})
            for cname, byd in cs.items():
                o[cname] = sum(byd.values()) / len(byd)
                o["dispatches"] = len(byd)
    return out


def summarize_trace(trace_dir, out_path, command, timed=(2, 12), kernel="k_march2<0, double>"):
    """Markdown summary of a rocprofv3 --kernel-trace --stats CSV run of the
    benchmark: the per-kernel statistics, and the durations of the headline
    kernel's dispatches in order, with their mean over the dispatches of the
    timed region (`timed`: first and one-past-last dispatch index; the default
    run's FP64 workload launches two pairs and a single step in its 5-step
    warm-up, then 10 pairs in its 20 timed steps)."""
    import csv
    import glob
    stats = []
    for path in glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True):
        with open(path) as fh:
            stats += list(csv.DictReader(fh))
    durs = []
    for path in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if kernel in r["Kernel_Name"]:
                    durs.append((int(r["Start_Timestamp"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
    durs.sort()
    us = [d for _, d in durs]
    a, b = timed
    lines = [f"# `{kernel}` on the 4096x1024 shock-interface workload: kernel trace of the benchmark", "",
             f"Command (repo root, on the GPU machine): `{command}`", "",
             f"Dispatches of `{kernel}`: {len(us)}; mean over all {sum(us) / max(len(us), 1):.2f} us.",
             f"Timed region of the FP64 run (dispatches {a + 1}..{b}): mean {sum(us[a:b]) / max(b - a, 1):.2f} us "
             f"over {len(us[a:b])} dispatches.", "",
             "Durations in order (us), first 120 dispatches:", "",
             " ".join(f"{x:.1f}" for x in us[:120]), "",
             "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    def num(r, *keys):
        for k in keys:
            if k in r and r[k] not in ("", None):
                return float(r[k])
        return float("nan")
    for r in sorted(stats, key=lambda r: -num(r, "TotalDurationNs"))[:25]:
        name = r.get("Name", "?")
        name = name[5:] if name.startswith("void ") else name
        name = name.replace("(anonymous namespace)::", "").split("(")[0]
        lines.append(f"| `{name}` | {int(num(r, 'Calls'))} | "
                     f"{num(r, 'TotalDurationNs') / 1e3:.1f} | {num(r, 'AverageNs') / 1e3:.2f} | "
                     f"{num(r, 'Percentage'):.2f} |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return sum(us[a:b]) / max(b - a, 1)


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
    # the served stream's arrival window: 60 s as configured
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    # the highest of 20, 25, 30 and 35 requests/s whose queue stayed bounded
    # (at 30 the offered load exceeds what the device achieves)
    ap.add_argument("--sustainable-rate", type=float, default=25.0)
    ap.add_argument("--light-rate", type=float, default=15.0)
    ap.add_argument("--summarize-profile", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "SQ_DIR"),
                    help="write the counter summary of three rocprofv3 --pmc runs of the profile command "
                         "to profiles/ and exit (no GPU)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_DIR",
                    help="print the mean per dispatch of every counter of rocprofv3 --pmc runs for the step "
                         "kernels and exit (no GPU)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "OUT_MD"),
                    help="write the markdown summary of a rocprofv3 kernel trace of this benchmark and exit")
    ap.add_argument("--trace-command", default="rocprofv3 --kernel-trace --stats --output-format csv -d TRACE_DIR "
                    "-o trace -- python3 bench.py --gpus 1 --steps 20 --warmup 5")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace[0], args.summarize_trace[1], args.trace_command))
        return
    if args.summarize_counters:
        print(json.dumps(summarize_counters(args.summarize_counters), indent=1))
        return
    if args.summarize_profile:
        out = summarize_profile(*args.summarize_profile, TRAFFIC_FILE)
        print(json.dumps(out, indent=1))
        return

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
    res = run_gpu(case, args.steps, args.warmup, args.noneq_every, log, args.steps_per_launch,
                  keep_macros=not args.no_fp32)
    rl = roofline(res, "fp64")

    extra = {}
    if not args.steps_per_launch and res["steps_per_launch"] == 2:
        # the same workload with one step per launch, for comparison
        r1 = run_gpu(case, args.steps, args.warmup, args.noneq_every, log, 1)
        rl1 = roofline(r1, "fp64")
        extra["fp64_one_step_per_launch"] = {"value": r1["value"], "ms_per_step": r1["ms_per_step"],
                                             "kernel_ms_per_step": round(r1["kernel_ms_avg"], 5),
                                             "core_clock_mhz_estimate": round(r1["clock_mhz"], 1), "roofline": rl1}
    if not args.no_fp32:
        case32 = W.shock_interface(precision="fp32")
        r32 = run_gpu(case32, args.steps, args.warmup, args.noneq_every, log, args.steps_per_launch,
                      keep_macros=True)
        rl32 = roofline(r32, "fp32")
        # the same steps in both storage precisions: FP32 against FP64
        err = macro_errors(r32.pop("macros"), res.pop("macros"), 1.4)
        extra["fp32_storage"] = {"value": r32["value"], "ms_per_step": r32["ms_per_step"],
                                 "steps_per_launch": r32["steps_per_launch"],
                                 "core_clock_mhz_estimate": round(r32["clock_mhz"], 1), "roofline": rl32,
                                 "speedup_vs_fp64": r32["value"] / res["value"],
                                 "rel_error_vs_fp64_after_timed_steps": {
                                     "steps": args.warmup + args.steps, "L1_Linf": err,
                                     "max": max(max(v) for v in err.values()),
                                     "velocity_denominator": "flow speed"}}
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
                                     label="offered load as specified (overloaded), first come first served by "
                                           "memory, stopped at the end of arrivals")
        extra["served_latency_policy"] = run_served(
            args.serve_rate, args.serve_seconds, log, drain=False, policy="latency",
            label="offered load as specified (overloaded), resident work bounded by a 2 s latency target, "
                  "smallest work first, shed beyond 4 s of expected wait; stopped at the end of arrivals")
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
        "steps_wall_ms_per_step": round(1e3 * res["steps_wall_s"] / args.steps, 5),
        "noneq_star_ms": round(res["noneq_ms"], 4),
        "noneq_star_passes_in_timed_region": res["noneq_passes_in_region"],
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
