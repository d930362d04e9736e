"""Host-side tests of the serving scheduler (paper_1305_4736_amd/serve.py)
with a stand-in for the library's batches: first come, first served within a
precision, the memory budget never exceeded and never overtaken, a full batch
letting the other precision pass, every request stepped exactly its budget,
every request answered once, a device allocation that fails although the
budget allows it (the request waits; the budget shrinks to what fit), a slot
the device flags non-finite (failed, not completed, out of the latencies),
and the latency policy (resident work bounded, smallest work first,
shedding)."""
import numpy as np
import pytest

from paper_1305_4736_amd import mrtfd, serve
from paper_1305_4736_amd import workloads as W


class FakeBatch:
    """Slots with step budgets; records admissions and the resident bytes."""

    def __init__(self, capacity, precision, limiter, ledger):
        self.capacity, self.precision = capacity, precision
        self.slots = {}
        self.ledger = ledger
        self.flags = np.zeros(capacity, dtype=np.int32)
        self.poison = ledger.get("poison", set())     # request keys whose solve goes non-finite

    def add(self, p, rho, ux, uy, T, nsteps):
        assert rho.shape == (p["ny"], p["nx"])
        k = min(set(range(self.capacity)) - set(self.slots))
        self.slots[k] = {"left": nsteps, "done": 0, "fp": mrtfd.footprint(p), "nsteps": nsteps,
                         "key": (self.precision, p["nx"], p["ny"], nsteps)}
        self.flags[k] = 0
        self.ledger["resident"] += self.slots[k]["fp"]
        self.ledger["peak"] = max(self.ledger["peak"], self.ledger["resident"])
        self.ledger["admitted"].append((self.precision, p["nx"], p["ny"], nsteps))
        return k

    def step(self, n):
        self.ledger.setdefault("ticks", []).append(sum(s["left"] > 0 for s in self.slots.values()))
        for k, s in self.slots.items():
            d = min(n, s["left"])
            s["left"] -= d
            s["done"] += d
            if d and s["key"] in self.poison:
                self.flags[k] = 1

    def remaining(self, k):
        return self.slots[k]["left"]

    def steps_done(self, k):
        return self.slots[k]["done"]

    def macros(self, k):
        return tuple(np.full((1, 2), float(k)) for _ in range(4))

    def remove(self, k):
        s = self.slots.pop(k)
        assert s["done"] == s["nsteps"] or s["key"] in self.poison
        self.ledger["resident"] -= s["fp"]
        self.ledger["finished"] += 1

    def sync(self):
        pass

    def status(self):
        if self.flags.any():
            err = mrtfd.NonFiniteError(mrtfd.ENONFINITE, "flagged")
            err.flags = self.flags.copy()
            self.flags[:] = 0
            raise err
        return self.flags.copy()

    def close(self):
        pass


def make_server(capacity, budget, ledger, steps_per_tick=300):
    factory = lambda cap, prec, lim: FakeBatch(cap, prec, lim, ledger)
    return serve.Server(capacity=capacity, steps_per_tick=steps_per_tick, reserve_bytes=0, keep_results=True,
                        batch_factory=factory, memory=(budget, 1 << 40))


def small_stream(n, seed):
    reqs = W.serve_stream(rate=1000.0, duration=10.0, seed=seed, log_lo=16, log_hi=48, max_requests=n)
    assert len(reqs) == n
    return reqs


def ledger():
    return {"resident": 0, "peak": 0, "admitted": [], "finished": 0}


def key(spec):
    p = spec["params"]
    return (p["precision"], p["nx"], p["ny"], spec["nsteps"])


def test_fifo_and_memory_budget():
    reqs = small_stream(40, seed=5)
    fps = [mrtfd.footprint(s["params"]) for _, s in reqs]
    budget = 3 * sorted(fps)[len(fps) // 2]       # about three requests resident at a time
    assert budget >= max(fps)
    led = ledger()
    with make_server(capacity=64, budget=budget, ledger=led) as srv:
        rep = srv.run(reqs, realtime=False, drain=True)
    assert rep["completed"] == rep["admitted"] == len(reqs) and rep["backlog"] == 0
    assert led["finished"] == len(reqs) and led["resident"] == 0
    assert led["peak"] <= budget and rep["max_resident_bytes"] <= budget
    # no full batch: admissions follow arrival order across both precisions
    assert led["admitted"] == [key(s) for _, s in reqs]
    assert sorted(rep["results"]) == list(range(len(reqs)))
    assert all(lat >= 0.0 for lat in (rep["p50_s"], rep["p99_s"]))


def test_full_batch_lets_the_other_precision_pass():
    reqs = small_stream(30, seed=11)
    led = ledger()
    with make_server(capacity=1, budget=1 << 40, ledger=led, steps_per_tick=100) as srv:
        rep = srv.run(reqs, realtime=False, drain=True)
    assert rep["completed"] == len(reqs) and led["finished"] == len(reqs)
    assert rep["max_active"] <= 2
    # first come, first served within each precision
    for prec in ("fp32", "fp64"):
        assert [a for a in led["admitted"] if a[0] == prec] == [key(s) for _, s in reqs
                                                                 if s["params"]["precision"] == prec]
    # a request waiting for its (full) batch does not hold back later
    # requests of the other precision: some of them are admitted first
    keys = [key(s) for _, s in reqs]
    assert len(set(keys)) == len(keys)
    pos = {k: n for n, k in enumerate(led["admitted"])}
    passed = [(i, j) for i in range(len(keys)) for j in range(i + 1, len(keys))
              if keys[i][0] != keys[j][0] and pos[keys[j]] < pos[keys[i]]]
    assert passed


def test_stop_at_end_of_arrivals_reports_backlog():
    reqs = small_stream(20, seed=3)
    fps = [mrtfd.footprint(s["params"]) for _, s in reqs]
    led = ledger()
    with make_server(capacity=64, budget=max(fps), ledger=led, steps_per_tick=1) as srv:
        rep = srv.run(reqs, realtime=False, drain=False, duration=0.0)
    # one admission round, one tick: requests are left waiting or resident
    assert rep["completed"] + rep["resident_at_end"] + rep["backlog"] == len(reqs)
    assert rep["backlog"] > 0


@pytest.mark.parametrize("seed", [13054737])
def test_request_recipe(seed):
    reqs = W.serve_stream(rate=200.0, duration=2.0, seed=seed)
    kinds = {s["kind"] for _, s in reqs}
    precs = {s["params"]["precision"] for _, s in reqs}
    assert kinds == {"quadrant", "couette"} and precs == {"fp32", "fp64"}
    for t, s in reqs:
        p = s["params"]
        assert 0.0 <= t < 2.0 and 64 <= p["nx"] <= 2048 and 64 <= p["ny"] <= 2048
        assert 200 <= s["nsteps"] <= 5000
    ts = [t for t, _ in reqs]
    assert ts == sorted(ts) and 300 <= len(reqs) <= 500     # Poisson, mean 400


class TightBatch(FakeBatch):
    """A device that holds less than the budget: adds fail with ENOMEM once
    the resident bytes would pass `device_bytes`."""

    def __init__(self, capacity, precision, limiter, ledger, device_bytes):
        super().__init__(capacity, precision, limiter, ledger)
        self.device_bytes = device_bytes

    def add(self, p, rho, ux, uy, T, nsteps):
        if self.ledger["resident"] + mrtfd.footprint(p) > self.device_bytes:
            self.ledger["refused"] += 1
            raise mrtfd.MRTFDError(mrtfd.ENOMEM, "cannot allocate")
        return super().add(p, rho, ux, uy, T, nsteps)


def test_allocation_failure_waits_and_shrinks_the_budget():
    reqs = small_stream(40, seed=5)
    led = dict(ledger(), refused=0)
    fps = sorted(mrtfd.footprint(s["params"]) for _, s in reqs)
    device = sum(fps[-4:])                       # room for about four of them
    factory = lambda cap, prec, lim: TightBatch(cap, prec, lim, led, device)
    srv = serve.Server(capacity=64, steps_per_tick=300, reserve_bytes=0, keep_results=True,
                       batch_factory=factory, memory=(1 << 40, 1 << 40))
    rep = srv.run(reqs, realtime=False)
    assert led["refused"] > 0                    # the budget alone would have admitted more
    assert led["peak"] <= device
    assert rep["completed"] == len(reqs) == led["finished"]
    assert sorted(rep["results"]) == list(range(len(reqs)))


def test_requests_that_cannot_fit_alone_are_rejected():
    # one request larger than the device: refused by the device with nothing
    # resident, it is rejected instead of waiting forever; the rest complete
    reqs = small_stream(12, seed=6)
    fps = [mrtfd.footprint(s["params"]) for _, s in reqs]
    big = max(range(len(reqs)), key=lambda k: fps[k])
    second = sorted(fps)[-2]
    device = (second + fps[big]) // 2            # every request fits alone but the largest
    assert second <= device < fps[big]
    led = dict(ledger(), refused=0)
    factory = lambda cap, prec, lim: TightBatch(cap, prec, lim, led, device)
    srv = serve.Server(capacity=64, steps_per_tick=300, reserve_bytes=0, keep_results=True,
                       batch_factory=factory, memory=(1 << 40, 1 << 40))
    rep = srv.run(reqs, realtime=False)
    assert rep["rejected"] == 1 and big not in rep["results"]
    assert rep["completed"] == len(reqs) - 1
    # and by the budget alone, before any allocation
    led = ledger()
    srv = make_server(64, device, led)
    rep = srv.run(reqs, realtime=False)
    assert rep["rejected"] == 1 and rep["completed"] == len(reqs) - 1


def test_flagged_request_fails_and_is_left_out():
    reqs = small_stream(16, seed=7)
    bad = {key(reqs[3][1]), key(reqs[9][1])}
    led = dict(ledger(), poison=bad)
    with make_server(capacity=64, budget=1 << 40, ledger=led, steps_per_tick=100) as srv:
        rep = srv.run(reqs, realtime=False, drain=True)
    assert rep["failed"] == 2 and rep["failed_requests"] == [3, 9]
    assert rep["completed"] == len(reqs) - 2 and 3 not in rep["results"] and 9 not in rep["results"]
    # their slots were freed at once (they did not run their whole budget)
    assert led["resident"] == 0 and led["finished"] == len(reqs)


def test_non_finite_result_fails():
    # a result the flag did not catch (the last step's output) is checked on the host
    reqs = small_stream(6, seed=8)

    class NaNBatch(FakeBatch):
        def macros(self, k):
            out = super().macros(k)
            if self.slots[k]["key"] == key(reqs[2][1]):
                out[0][0, 0] = np.nan
            return out

    led = ledger()
    srv = serve.Server(capacity=64, steps_per_tick=300, reserve_bytes=0, keep_results=True,
                       batch_factory=lambda cap, prec, lim: NaNBatch(cap, prec, lim, led), memory=(1 << 40, 1 << 40))
    rep = srv.run(reqs, realtime=False)
    assert rep["failed_requests"] == [2] and rep["completed"] == 5


def test_latency_policy_bounds_resident_work_and_sheds():
    reqs = small_stream(60, seed=9)
    w = lambda s: s["params"]["nx"] * s["params"]["ny"] * s["nsteps"]
    works = sorted(w(s) for _, s in reqs)
    # a rate at which a tick of 100 steps is "1 s": the target holds about
    # the median request, the shedding bound a few of them
    rate = float(np.median(works))
    led = ledger()
    srv = serve.Server(capacity=64, steps_per_tick=100, reserve_bytes=0, keep_results=True,
                       batch_factory=lambda cap, prec, lim: FakeBatch(cap, prec, lim, led),
                       memory=(1 << 40, 1 << 40), policy="latency", latency_target_s=1.0,
                       shed_after_s=6.0, rate_guess=rate, measure_rate=False)
    rep = srv.run(reqs, realtime=False)
    # every request is answered once: completed, or shed
    assert rep["completed"] + rep["shed"] == len(reqs) and rep["failed"] == 0
    assert rep["shed"] > 0 and set(rep["shed_requests"]).isdisjoint(rep["results"])
    # the shed ones are the largest (smallest work first)
    done_w = [w(reqs[i][1]) for i in rep["results"]]
    shed_w = [w(reqs[i][1]) for i in rep["shed_requests"]]
    assert np.median(shed_w) > np.median(done_w)
    # admitted in order of work within the first admission round
    first = [a for a in led["admitted"]][:3]
    assert [a[1] * a[2] * a[3] for a in first] == sorted(a[1] * a[2] * a[3] for a in first)
