"""GPU test of the serving loop (continuous batching).

A small stream of requests of different kinds (Riemann quadrants, thermal
Couette flows), grid sizes, step counts and precisions is served, under
each admission policy, with requests joining while others are running and
slots being reused.  Each
served result must equal the same request run alone (bitwise, the per-node
arithmetic does not depend on the mix) and match the FP64 oracle (1e-11
relative for FP64 storage, 2e-5 for FP32 storage).
"""
import numpy as np
import pytest

from parity import TOL, assert_parity
from paper_1305_4736_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_4736_amd import mrtfd, serve
    return mrtfd, serve


def small_stream(n=14, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for k in range(n):
        t += rng.exponential(0.002)
        spec = W.serve_request(rng, k, log_lo=8, log_hi=48)
        spec["nsteps"] = int(rng.integers(5, 60))
        out.append((t, spec))
    return out


@pytest.mark.parametrize("policy", ["fifo", "latency"])
def test_served_results_equal_alone_and_oracle(lib, orc, policy):
    mrtfd, serve = lib
    reqs = small_stream()
    # capacity 3 per precision: later requests wait for slots and reuse them;
    # the latency policy admits smallest work first within its bound
    with serve.Server(capacity=3, steps_per_tick=7, keep_results=True, reserve_bytes=0, policy=policy) as srv:
        rep = srv.run(reqs, realtime=True)
    assert rep["completed"] == len(reqs) and rep["backlog"] == 0
    assert rep["failed"] == 0 and rep["shed"] == 0
    assert rep["max_active"] <= 6 and rep["ticks"] > 3
    assert np.isfinite(rep["p50_s"]) and rep["p99_s"] >= rep["p50_s"]
    for i, (t, spec) in enumerate(reqs):
        case = W.spec_case(spec)
        p = case["params"]
        with mrtfd.Solver(p) as s:
            s.init(case["rho"], case["ux"], case["uy"], case["T"])
            s.step(spec["nsteps"])
            alone = s.macros()
        served = rep["results"][i]
        for a, b in zip(alone, served):
            assert np.array_equal(a, b), spec["name"]
        if i % 3 == 0:
            fo = orc.run(p, case["rho"], case["ux"], case["uy"], case["T"], spec["nsteps"])
            assert_parity(served, orc.macros(p, fo), TOL[p["precision"]], 1.4, spec["name"])


def test_failed_request_is_unphysical_for_the_oracle_too(lib, orc):
    """The request the overloaded served streams report as failed, request
    2041 of the 60-s stream at 200 requests/s (a quadrant problem on
    135 x 175 in FP64 storage, 2969 steps; the stream's specs do not depend
    on its rate), fails in the scheme, not in the GPU path: run alone, the
    GPU state and the oracle's agree at the FP64 bar after 900 steps, both
    physical; within the next 50 steps the oracle's temperature goes
    negative at some node (from step 917 to 944, then positive again) and
    the GPU flags the run."""
    mrtfd, _ = lib
    spec = W.serve_stream(rate=200.0, duration=60.0)[2041][1]
    assert (spec["kind"], spec["params"]["nx"], spec["params"]["ny"]) == ("quadrant", 135, 175)
    case = W.spec_case(spec)
    p = dict(case["params"], precision="fp64")
    print("[serve] request 2041 alone: GPU and oracle to step 900, then 50 more", flush=True)
    with mrtfd.Solver(p) as s:
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(900)
        s.sync()                                  # nothing flagged yet
        m900 = s.macros()
        s.step(50)
        with pytest.raises(mrtfd.NonFiniteError):
            s.sync()
    fo = orc.run(p, case["rho"], case["ux"], case["uy"], case["T"], 900)
    o900 = orc.macros(p, fo)
    assert min(np.min(m900[3]), np.min(o900[3])) > 0.0
    errs = assert_parity(m900, o900, TOL["fp64"], 1.4, "request 2041 at step 900")
    tmin = []
    for _ in range(50):
        fo = orc.advance(p, fo, 1)
        tmin.append(float(np.min(orc.macros(p, fo)[3])))
    print(f"[serve] request 2041 at step 900: {errs}; oracle T min over steps 901-950: {min(tmin):.3e}", flush=True)
    assert min(tmin) <= 0.0
