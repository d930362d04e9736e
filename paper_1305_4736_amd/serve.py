"""Serving loop: continuous batching of MRT-FD solves on one GPU.

Requests (a grid, an initial state, rates, boundaries, a step count and a
storage precision) arrive over time.  The loop

  * admits waiting requests while device memory and slots allow: a
    request's state (two padded state buffers) must fit in the free HBM
    left after a reserve, under an optional cap on resident bytes.  Two
    admission policies:
      - "fifo": first come, first served, by memory alone;
      - "latency": the resident work (node-updates still to do) is kept
        within what the device turns over in `latency_target_s` at the
        throughput measured so far, waiting requests are admitted smallest
        work first, and a request whose expected wait (the work resident and
        queued ahead of it, over that throughput) exceeds `shed_after_s` is
        shed (answered with a refusal) instead of queued;
  * keeps every admitted request's state resident as a slot of one of two
    batches (FP32 storage, FP64), each slot with its own step budget; by
    default each batch has a stream of its own, so the two overlap on the
    device;
  * every tick, advances both batches by `steps_per_tick` launches: all
    resident requests progress together, requests that arrived during the
    previous tick join as soon as they are admitted, and a request that uses
    up its budget stops stepping inside the tick;
  * hands finished requests their (rho, u_x, u_y, T) on the host, records the
    latency (arrival to result on the host) and frees their slot; a request
    whose slot the device flagged (a node reached rho <= 0, T <= 0 or NaN)
    or whose result is not finite is counted as failed, its slot freed, and
    it enters neither the completed count nor the latency percentiles.

All stepping runs in the library's batched kernels; this module only
schedules.  The report gives p50 / p99 latency beside offered and achieved
node-updates per second.
"""
from __future__ import annotations

import collections
import contextlib
import time

import numpy as np

from . import mrtfd
from . import workloads as W


class Server:
    """`batch_factory(capacity, precision, limiter)`, `memory` = (free, total)
    bytes and `materialize(spec)` replace the library batches, the device
    memory query and the device-side field construction (scheduling tests run
    them on the host)."""

    def __init__(self, capacity=2048, steps_per_tick=50, reserve_bytes=8 << 30, max_resident_bytes=None,
                 limiter="mc", stream=None, keep_results=False, batch_factory=None, memory=None,
                 materialize=None, overlap_nodes=1 << 25, policy="fifo", latency_target_s=2.0,
                 shed_after_s=None, rate_guess=2.5e10, measure_rate=True):
        if policy not in ("fifo", "latency"):
            raise ValueError(f"unknown admission policy {policy!r}")
        self.policy = policy
        self.latency_target = float(latency_target_s)
        self.shed_after = float(shed_after_s) if shed_after_s is not None else 2.0 * self.latency_target
        # node-updates/s assumed until the first ticks have measured it (or
        # throughout, with measure_rate=False)
        self.rate_guess = float(rate_guess)
        self.measure_rate = bool(measure_rate)
        self.streams = None
        if batch_factory is None:
            import torch
            device = torch.device("cuda", torch.cuda.current_device())
            if stream is not None:
                self.streams = {"fp32": stream, "fp64": stream}
            else:
                # default priority, like every stream here
                self.streams = {"fp32": torch.cuda.current_stream(), "fp64": torch.cuda.Stream(device=device)}
            batch_factory = lambda cap, prec, lim: mrtfd.Batch(cap, precision=prec, limiter=lim,
                                                              stream=self.streams[prec])
            if materialize is None:
                materialize = lambda spec: W.materialize(spec, torch, device=device)
        self.materialize = materialize if materialize is not None else W.materialize
        self.memory = memory
        self.batches = {p: batch_factory(capacity, p, limiter) for p in ("fp32", "fp64")}
        self.capacity = capacity
        self.k = int(steps_per_tick)
        self.reserve = int(reserve_bytes)
        self.cap_bytes = max_resident_bytes
        self.keep_results = keep_results
        # the two batches overlap on the device while either has fewer active
        # nodes than this; two heavy batches take turns (each one's persistent
        # launches are sized to fill the device, and sharing it cost 10 % of
        # the overloaded stream's throughput)
        self.overlap_nodes = int(overlap_nodes)

    def _on(self, precision):
        """Context in which a request's device fields are made: its batch's
        stream, which then reads them in order."""
        if self.streams is None:
            return contextlib.nullcontext()
        import torch
        return torch.cuda.stream(self.streams[precision])

    def close(self):
        for b in self.batches.values():
            b.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, stream_reqs, duration=None, drain=True, log=None, realtime=True):
        """Serve [(arrival_s, spec), ...] (sorted).  With realtime=False every
        request arrives at t = 0.  Returns a report dict (and results if
        keep_results)."""
        reqs = sorted(stream_reqs, key=lambda r: r[0])
        free0, total = self.memory if self.memory is not None else mrtfd.device_memory()
        budget = free0 - self.reserve
        if self.cap_bytes is not None:
            budget = min(budget, int(self.cap_bytes))
        budget0 = budget            # the host's bound; `budget` also learns what the device holds
        pending = collections.deque()
        active = {}                 # (precision, slot) -> request record
        resident = 0
        nxt = 0
        lat, done_nodeupd, results, admitted, ticks = [], 0.0, {}, 0, 0
        rejected = []               # requests the device cannot hold even alone
        shed = []                   # requests refused by the latency policy
        failed = []                 # requests whose solve went non-finite
        rate = None                 # measured node-updates/s (latency policy)
        work = lambda spec: spec["params"]["nx"] * spec["params"]["ny"] * spec["nsteps"]
        max_resident, max_active = 0, 0
        t0 = time.perf_counter()
        while True:
            now = time.perf_counter() - t0
            while nxt < len(reqs) and (not realtime or reqs[nxt][0] <= now):
                pending.append(nxt)
                nxt += 1
            # without draining, the run ends with the arrival window
            stop_admitting = duration is not None and now >= duration and not drain
            # admission.  fifo: first come, first served within each precision,
            # by free memory and free slots (a request whose batch is full is
            # passed by requests of the other precision; memory is never
            # overtaken).  latency: smallest work first, while the resident
            # work stays within what the device does in the latency target
            if pending and not stop_admitting:
                keep = collections.deque()
                full = {p: sum(1 for k in active if k[0] == p) >= self.capacity for p in self.batches}
                mem_blocked = False
                work_blocked = False
                if self.policy == "latency":
                    r = rate if rate else self.rate_guess
                    resident_work = sum(rec["nodes"] * self.batches[k[0]].remaining(k[1]) for k, rec in active.items())
                    order = sorted(pending, key=lambda i: (work(reqs[i][1]), i))
                    # shed requests that could not start within the bound:
                    # the work resident and queued ahead of them, over the rate
                    ahead = resident_work
                    keep_order = []
                    for i in order:
                        if ahead / r > self.shed_after:
                            shed.append(i)
                            continue
                        keep_order.append(i)
                        ahead += work(reqs[i][1])
                    pending = collections.deque(keep_order)
                while pending:
                    i = pending.popleft()
                    t_arr, spec = reqs[i]
                    if self.policy == "latency":
                        if work_blocked or (resident_work > 0 and resident_work + work(spec) > r * self.latency_target):
                            work_blocked = True
                            keep.append(i)
                            continue
                    p = spec["params"]
                    fp = mrtfd.footprint(p)
                    if fp > budget0:
                        rejected.append(i)      # larger than the whole budget: would wait forever
                        continue
                    # with nothing resident a request is always tried (the
                    # device decides); otherwise it waits for room
                    fits = resident == 0 or resident + fp <= budget
                    if mem_blocked or full[p["precision"]] or not fits:
                        mem_blocked = mem_blocked or (not fits and not full[p["precision"]])
                        keep.append(i)
                        continue
                    b = self.batches[p["precision"]]
                    try:
                        with self._on(p["precision"]):
                            slot = b.add(p, *self.materialize(spec), nsteps=spec["nsteps"])
                    except mrtfd.MRTFDError as e:
                        if e.code != mrtfd.ENOMEM:
                            raise
                        if resident == 0:
                            rejected.append(i)  # does not fit even alone
                            continue
                        # the device holds less than the footprints add up to
                        # (allocator rounding and caching): the request waits,
                        # and what is resident now becomes the budget
                        budget = min(budget, resident)
                        mem_blocked = True
                        keep.append(i)
                        continue
                    active[(p["precision"], slot)] = {"i": i, "t": t_arr if realtime else 0.0, "fp": fp,
                                                      "nodes": p["nx"] * p["ny"], "steps": spec["nsteps"]}
                    if self.policy == "latency":
                        resident_work += work(spec)
                    resident += fp
                    budget = max(budget, resident)
                    admitted += 1
                    full[p["precision"]] = sum(1 for k in active if k[0] == p["precision"]) >= self.capacity
                pending = keep
            max_resident = max(max_resident, resident)
            max_active = max(max_active, len(active))
            if not active:
                if nxt >= len(reqs) and not pending:
                    break
                if stop_admitting:
                    break
                if realtime and nxt < len(reqs):
                    time.sleep(max(0.0, min(reqs[nxt][0] - (time.perf_counter() - t0), 0.002)))
                continue
            # one tick: every resident request advances (up to its budget)
            nodes = {p: sum(r["nodes"] for k, r in active.items() if k[0] == p) for p in self.batches}
            busy = [p for p in self.batches if nodes[p] > 0]
            turns = self.streams is not None and len(busy) == 2 and min(nodes.values()) >= self.overlap_nodes
            latency = self.policy == "latency" and self.measure_rate
            before = {k: self.batches[k[0]].steps_done(k[1]) for k in active} if latency else None
            t_tick = time.perf_counter()
            for i, prec in enumerate(busy):
                if turns and i > 0:
                    self.streams[prec].wait_stream(self.streams[busy[i - 1]])
                self.batches[prec].step(self.k)
            for b in self.batches.values():
                b.sync()
            ticks += 1
            tick_s = time.perf_counter() - t_tick
            if latency and tick_s > 0:
                moved = sum(rec["nodes"] * (self.batches[k[0]].steps_done(k[1]) - before[k]) for k, rec in active.items())
                if moved > 0:
                    r_tick = moved / tick_s
                    rate = r_tick if rate is None else 0.8 * rate + 0.2 * r_tick
            # slots the device flagged since the last tick (flags are cleared
            # by the check, so they are read every tick)
            flagged = set()
            for prec, b in self.batches.items():
                try:
                    b.status()
                except mrtfd.NonFiniteError as e:
                    flagged |= {(prec, int(k)) for k in np.nonzero(np.asarray(e.flags))[0]}
            # finished requests: results to the host, slots freed; flagged
            # requests end as failed at once
            finished = [key for key in active if key in flagged or self.batches[key[0]].remaining(key[1]) == 0]
            for key in finished:
                b = self.batches[key[0]]
                rec = active.pop(key)
                ok = key not in flagged
                out = b.macros(key[1]) if ok else None
                if ok and not all(np.all(np.isfinite(np.asarray(q))) for q in out):
                    ok = False
                if ok:
                    t_done = time.perf_counter() - t0
                    lat.append(t_done - rec["t"])
                    done_nodeupd += rec["nodes"] * rec["steps"]
                    if self.keep_results:
                        results[rec["i"]] = out
                else:
                    failed.append(rec["i"])
                    done_nodeupd += rec["nodes"] * b.steps_done(key[1])
                b.remove(key[1])
                resident -= rec["fp"]
            if log and ticks % 20 == 0:
                log(f"[serve] t={time.perf_counter() - t0:.1f}s active={len(active)} pending={len(pending)} "
                    f"done={len(lat)}")
            if stop_admitting:
                break
        elapsed = time.perf_counter() - t0
        # work done by requests still resident (partial)
        partial = sum(rec["nodes"] * self.batches[k[0]].steps_done(k[1]) for k, rec in active.items())
        offered = sum(s["params"]["nx"] * s["params"]["ny"] * s["nsteps"] for _, s in reqs)
        span = max(reqs[-1][0], 1e-9) if (reqs and realtime) else None
        lat_a = np.array(lat) if lat else np.array([np.nan])
        report = {
            "policy": self.policy,
            "requests": len(reqs), "admitted": admitted, "completed": len(lat), "rejected": len(rejected),
            "shed": len(shed), "failed": len(failed),
            "backlog": len(pending) + (len(reqs) - nxt), "resident_at_end": len(active),
            "latency_over": "completed requests only",
            "p50_s": float(np.percentile(lat_a, 50)), "p99_s": float(np.percentile(lat_a, 99)),
            "mean_s": float(np.mean(lat_a)), "elapsed_s": elapsed, "ticks": ticks,
            "steps_per_tick": self.k,
            "achieved_node_updates_per_s": (done_nodeupd + partial) / elapsed,
            "offered_node_updates_per_s": (offered / span) if span else None,
            "max_resident_bytes": max_resident, "max_active": max_active,
            "hbm_budget_bytes": budget,
        }
        if self.policy == "latency":
            report.update({"latency_target_s": self.latency_target, "shed_after_s": self.shed_after,
                           "measured_rate": rate})
        # indices into the stream: failures are few and named in every
        # report; shed requests can run to thousands
        report["failed_requests"] = sorted(failed)
        if self.keep_results:
            report["results"] = results
            report["shed_requests"] = sorted(shed)
        return report
