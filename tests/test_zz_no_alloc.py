"""The no-allocation solve (mrtfd_solve_noalloc) against the allocating
entry points (mrtfd_create, mrtfd_init, mrtfd_step, mrtfd_macros) on the
same inputs: bit for bit (the same kernels on the same bytes), which is
within the FP64 bar of 1e-11 and the FP32 bar of 2e-5.  Calls follow one
another on one GPU, each smaller than the one before, so every call reuses
the array the previous one left behind; the sizes beyond the array are
refused with MRTFD_EINVAL."""
import numpy as np
import pytest

from paper_1305_4736_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P, E, O = W.bc("periodic"), W.bc("equilibrium", 1.1, 0.05, -0.02, 0.9), W.bc("outflow")
WL, WH = W.bc("wall", 1.0, 0.0, 0.0, 1.0), W.bc("wall", 1.0, 0.15, 0.0, 1.05)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_4736_amd import mrtfd
    return mrtfd


def dev_fields(case):
    d = torch.device("cuda:0")
    return [torch.tensor(case[k], dtype=torch.float64, device=d) for k in ("rho", "ux", "uy", "T")]


def allocating(lib, case, n):
    with lib.Solver(case["params"]) as s:
        s.init(*dev_fields(case))
        s.step(n)
        s.sync()
        return s.macros()


def no_alloc(lib, case, n):
    print(f"[no-alloc] {case['params']['nx']}x{case['params']['ny']} {case['params']['precision']} {n} steps",
          flush=True)
    out = lib.solve_noalloc(case["params"], *dev_fields(case), n)
    torch.cuda.synchronize()
    return tuple(o.cpu().numpy() for o in out)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_no_alloc_equals_the_allocating_path(lib, precision):
    cases = [
        # two steps per launch by default (4 rows or more per pair band)
        (W.random_smooth(400, 300, seed=41, bcs=[E, O, P, P], jumps=True, precision=precision), 30),
        # walls along y, refilled inside the step kernels
        (W.random_smooth(130, 61, seed=42, bcs=[P, P, WL, WH], jumps=True, precision=precision), 21),
        # walls along x, refilled by a launch after each step
        (W.random_smooth(67, 13, seed=43, bcs=[WL, WH, O, O], jumps=True, precision=precision), 17),
    ]
    for case, n in cases:
        got = no_alloc(lib, case, n)
        ref = allocating(lib, case, n)
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), (case["name"], precision)


def test_no_alloc_refuses_grids_beyond_the_array(lib):
    case = W.random_smooth(600, 600, precision="fp64")
    with pytest.raises(lib.MRTFDError) as e:
        lib.solve_noalloc(case["params"], *dev_fields(case), 1)
    assert e.value.code == lib.EINVAL and "no-allocation" in str(e.value)
    # and the array still serves the next call
    small = W.random_smooth(50, 20, seed=44)
    assert all(np.array_equal(a, b) for a, b in zip(no_alloc(lib, small, 5), allocating(lib, small, 5)))
