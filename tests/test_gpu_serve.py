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
