"""GPU parity: the gfx950 path (through the C ABI) against the FP64 oracle,
element by element on the same seeded inputs.

Bars: FP64 storage within 1e-11 relative (L1 and Linf in rho, u, T and in
f itself); FP32 storage within 2e-5 relative in rho, u, T.

Cases: random smooth and discontinuous states on ragged grids that span
several 64 x 4 thread blocks, with every boundary kind and limiter, the
correction on and off; degenerate grids (one row, one column, one fluid row
between walls); the Sod tube in full (3600 steps); Couette flow at 200
nodes; the heavy/light shock-interface problem on a reduced grid, and at its
full 4096 x 1024 size checked on windows the oracle can compute on its own
(the explicit stencil reaches two nodes per step, so a window's interior
farther than 2n + 2 nodes from its cut edges is exact after n steps).
"""
import math

import numpy as np
import pytest

from parity import TOL, assert_parity, f_rel, window_params
from paper_1305_4736_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_4736_amd import mrtfd   # raises if the library is not built
    return mrtfd


def run_gpu(lib, case, nsteps=None, precision=None):
    p = dict(case["params"])
    if precision:
        p["precision"] = precision
    n = case["nsteps"] if nsteps is None else nsteps
    with lib.Solver(p) as s:
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(n)
        s.sync()
        return s.macros(), s.get_f()


def run_orc(orc, case, nsteps=None):
    p = case["params"]
    n = case["nsteps"] if nsteps is None else nsteps
    f = orc.run(p, case["rho"], case["ux"], case["uy"], case["T"], n)
    return orc.macros(p, f), f


def gamma_of(case):
    b = case["params"]["b"]
    return (b + 2.0) / b


def check_case(lib, orc, case, precision="fp64", nsteps=None, f_tol=None):
    print(f"[parity] {case['name']} {precision} nsteps={nsteps or case['nsteps']}", flush=True)
    mg, fg = run_gpu(lib, case, nsteps, precision)
    mo, fo = run_orc(orc, case, nsteps)
    errs = assert_parity(mg, mo, TOL[precision], gamma_of(case), case["name"])
    if precision == "fp64":
        assert f_rel(fg, fo) <= (f_tol or TOL["fp64"])
    return errs


P, E, O = W.bc("periodic"), W.bc("equilibrium", 1.1, 0.05, -0.02, 0.9), W.bc("outflow")
WL, WH = W.bc("wall", 1.0, 0.0, 0.0, 1.0), W.bc("wall", 1.0, 0.15, 0.0, 1.05)
BC_SETS = {
    "periodic": [P, P, P, P],
    "eq_x_periodic_y": [E, W.bc("equilibrium", 0.8, -0.1, 0.0, 1.2), P, P],
    "outflow_all": [O, O, O, O],
    "inflow_outflow": [E, O, P, P],
    "walls_y": [P, P, WL, WH],
    "walls_x": [W.bc("wall", 1.0, 0.0, 0.0, 1.0), W.bc("wall", 1.0, 0.0, -0.1, 1.0), P, P],
    "outflow_x_eq_y": [O, O, E, W.bc("equilibrium", 1.0, 0.0, 0.1, 1.0)],
}


@pytest.mark.parametrize("bcs", sorted(BC_SETS))
@pytest.mark.parametrize("limiter", ["mc", "minmod"])
def test_random_ragged_fp64(lib, orc, bcs, limiter):
    case = W.random_smooth(67, 13, seed=sum(map(ord, bcs)), bcs=BC_SETS[bcs], limiter=limiter,
                           jumps=True, nsteps=25)
    check_case(lib, orc, case)


@pytest.mark.parametrize("limiter", ["lw", "upwind"])
def test_other_limiters_fp64(lib, orc, limiter):
    case = W.random_smooth(70, 9, seed=3, bcs=BC_SETS["inflow_outflow"], limiter=limiter, nsteps=20)
    check_case(lib, orc, case)


def anisotropic(case, ratio=1.6):
    # dy = ratio dx, dt within the unsplit Courant bound of the smaller spacing
    p = dict(case["params"])
    p.update(dy=ratio * p["dx"], dt=0.3 * p["dx"] / 6.0)
    return dict(case, params=p, name=case["name"] + "_dy%.1fdx" % ratio)


@pytest.mark.parametrize("bcs", ["inflow_outflow", "walls_y", "walls_x", "outflow_x_eq_y"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_unequal_spacings(lib, orc, bcs, precision):
    # every other test has dy = dx: a spacing taken for the other axis (in the
    # Courant numbers or the velocity gradients of the correction) would pass
    # them; here dy = 1.6 dx, one and two steps per launch and in a batch
    case = anisotropic(W.random_smooth(130, 61, seed=31, bcs=BC_SETS[bcs], jumps=True, nsteps=20))
    check_case(lib, orc, case, precision)
    mo, _ = run_orc(orc, case)
    p = dict(case["params"], precision=precision)
    if bcs != "walls_x":
        with lib.Solver(p) as s:
            s.steps_per_launch = 2
            s.init(case["rho"], case["ux"], case["uy"], case["T"])
            s.step(20)
            s.sync()
            assert_parity(s.macros(), mo, TOL[precision], gamma_of(case), case["name"] + " fused")
    with lib.Batch(1, precision=precision) as b:
        k = b.add(p, case["rho"], case["ux"], case["uy"], case["T"], nsteps=20)
        b.step(20)
        assert_parity(b.macros(k), mo, TOL[precision], gamma_of(case), case["name"] + " batch")


def test_correction_off_fp64(lib, orc):
    case = W.random_smooth(40, 40, seed=12, bcs=BC_SETS["walls_y"], correction=False, nsteps=20)
    check_case(lib, orc, case)


@pytest.mark.parametrize("shape,bcs", [((1, 37), "periodic"), ((45, 1), "eq_x_periodic_y"),
                                       ((1, 1), "periodic"), ((5, 3), "walls_y"),
                                       ((3, 7), "walls_x"), ((2, 2), "outflow_all"),
                                       ((129, 4), "periodic"), ((64, 4), "inflow_outflow")])
def test_degenerate_and_block_edge_shapes_fp64(lib, orc, shape, bcs):
    case = W.random_smooth(shape[0], shape[1], seed=7, bcs=BC_SETS[bcs], nsteps=15)
    check_case(lib, orc, case)


@pytest.mark.parametrize("limiter", ["minmod", "mc"])
def test_sod_full_run_fp64(lib, orc, limiter):
    check_case(lib, orc, W.sod(limiter=limiter))


@pytest.mark.parametrize("pr", [0.5, 1.0, 2.0])
def test_couette_fp64(lib, orc, pr):
    case = W.couette(pr=pr, gamma=1.4)
    check_case(lib, orc, case, nsteps=3000)


def test_shock_interface_reduced_fp64(lib, orc):
    case = W.shock_interface(nx=384, ny=96, nsteps=120)
    check_case(lib, orc, case)


@pytest.mark.parametrize("precision", ["fp32"])
@pytest.mark.parametrize("which", ["sod", "random_walls", "random_outflow", "shock"])
def test_fp32_storage(lib, orc, precision, which):
    if which == "sod":
        case = W.sod()
    elif which == "random_walls":
        case = W.random_smooth(67, 13, seed=5, bcs=BC_SETS["walls_y"], jumps=True, nsteps=200)
    elif which == "random_outflow":
        case = W.random_smooth(67, 13, seed=6, bcs=BC_SETS["outflow_all"], jumps=True, nsteps=200)
    else:
        case = W.shock_interface(nx=384, ny=96, nsteps=120)
    check_case(lib, orc, case, precision=precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("star", [False, True])
def test_noneq(lib, orc, precision, star):
    case = W.random_smooth(67, 13, seed=21, bcs=BC_SETS["inflow_outflow"], jumps=True, nsteps=30)
    p = dict(case["params"], precision=precision)
    with lib.Solver(p) as s:
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(30)
        dg = s.noneq(star)
        fg = s.get_f()
    # oracle on the GPU's own state isolates the diagnostic from the stepping
    do = orc.noneq(case["params"], fg, star)
    scale = np.abs(do[4:]).max()
    assert np.abs(dg - do).max() <= 1e-11 * scale
    # and on the oracle's own trajectory (FP64 only: FP32 storage drifts by ~1e-6)
    if precision == "fp64":
        fo = orc.run(case["params"], case["rho"], case["ux"], case["uy"], case["T"], 30)
        do2 = orc.noneq(case["params"], fo, star)
        assert np.abs(dg - do2).max() <= 1e-10 * scale


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_checkpoint_resume_is_bitwise(lib, precision):
    case = W.random_smooth(67, 13, seed=2, bcs=BC_SETS["walls_y"], jumps=True)
    p = dict(case["params"], precision=precision)
    with lib.Solver(p) as s:
        assert s.state_planes == (20 if precision == "fp32" else 16)
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(10)
        st10 = s.get_state()
        s.step(10)
        st20 = s.get_state()
        f20 = s.get_f()
        s.set_state(st10)
        assert np.array_equal(s.get_state(), st10)
        s.step(10)
        assert np.array_equal(s.get_state(), st20)
        assert np.array_equal(s.get_f(), f20)
        assert s.steps_done == 10
        if precision == "fp64":
            # in FP64 storage the populations are the whole state
            s.set_f(st10)
            assert np.array_equal(s.get_f(), st10)
            s.step(10)
            assert np.array_equal(s.get_f(), f20)


def test_fp32_populations_carry_their_stored_conserved_moments(lib, orc):
    # get_f of FP32 storage gives populations whose conserved moments are the
    # stored FP64 ones; set_f of them stores those moments again
    case = W.random_smooth(67, 13, seed=4, bcs=BC_SETS["inflow_outflow"], jumps=True)
    p = dict(case["params"], precision="fp32")
    _, M, _, _ = orc.constants()
    with lib.Solver(p) as s:
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(7)
        st = s.get_state()
        f = s.get_f()
        c = np.einsum("ki,iyx->kyx", M[:4], f)
        assert np.abs(c - st[16:]).max() <= 1e-14 * np.abs(st[16:]).max()
        # the populations are the stored FP32 ones to within a few of their ulps
        assert np.abs(f - st[:16]).max() <= 8 * np.spacing(np.abs(st[:16]).astype(np.float32)).max()
        s.set_f(f)
        st2 = s.get_state()
        assert np.abs(st2[16:] - st[16:]).max() <= 1e-14 * np.abs(st[16:]).max()


def test_nonfinite_is_reported(lib):
    case = W.random_smooth(33, 9, seed=1)
    with lib.Solver(case["params"]) as s:
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(3)
        s.sync()
        f = s.get_f()
        f[:, 4, 17] = np.nan
        s.set_f(f)
        s.step(2)
        with pytest.raises(lib.NonFiniteError):
            s.sync()
        s.sync()    # the flag was cleared


def test_device_pointers(lib, orc):
    case = W.random_smooth(50, 20, seed=8, bcs=BC_SETS["inflow_outflow"], nsteps=12)
    dev = torch.device("cuda:0")
    fields = [torch.tensor(case[k], dtype=torch.float64, device=dev) for k in ("rho", "ux", "uy", "T")]
    with lib.Solver(case["params"]) as s:
        s.init(*fields)
        s.step(12)
        out = tuple(torch.empty((20, 50), dtype=torch.float64, device=dev) for _ in range(4))
        s.macros(out)
        torch.cuda.synchronize()
        mg = tuple(o.cpu().numpy() for o in out)
    mo, _ = run_orc(orc, case)
    assert_parity(mg, mo, TOL["fp64"])


# ----------------------------------------------------------------------------
# Full size of the large shock-interface workload (4096 x 1024), in the same
# launch configuration the benchmark times, checked on oracle windows.

def _window_case(case, x0, nxw, y0, nyw):
    ny, nx = case["rho"].shape
    rows = [(y0 + j) % ny for j in range(nyw)]
    sl = lambda a: a[rows][:, x0:x0 + nxw]
    p = window_params(case["params"], x0, nxw, y0, nyw, keep_x_lo=(x0 == 0), keep_x_hi=(x0 + nxw == nx))
    return p, sl


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shock_interface_full_size_windows(lib, orc, precision):
    nsteps = 12
    case = W.shock_interface(precision=precision)
    ny, nx = case["rho"].shape
    print(f"[parity] shock_interface full {nx}x{ny} {precision} {nsteps} steps", flush=True)
    with lib.Solver(case["params"]) as s:
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(nsteps)
        s.sync()
        mg = s.macros()
    margin = 2 * nsteps + 2
    # windows: inflow edge, interface crests, shock, outflow edge, across the y seam
    for x0, y0 in [(0, 100), (880, 0), (940, 250), (1000, 700), (4096 - 96, 500), (960, 1024 - 48)]:
        nxw, nyw = 96, 96
        p, sl = _window_case(case, x0, nxw, y0, nyw)
        fo = orc.run(p, sl(case["rho"]), sl(case["ux"]), sl(case["uy"]), sl(case["T"]), nsteps)
        mo = orc.macros(p, fo)
        xs = slice(0 if x0 == 0 else margin, nxw if x0 + nxw == nx else nxw - margin)
        ys = slice(margin, nyw - margin)
        gw = tuple(sl(m)[ys, xs] for m in mg)
        ow = tuple(m[ys, xs] for m in mo)
        assert_parity(gw, ow, TOL[precision], 1.4, f"window x0={x0} y0={y0}")


def test_state_buffers_of_2gib_and_more_use_the_tile_form(lib, orc):
    # a 4096 x 4200 FP64 grid holds 2.2 GB per state buffer: beyond the
    # row-marching form's 31-bit offsets, so the step runs the LDS-tile form
    nsteps = 6
    case = W.shock_interface(nx=4096, ny=4200, x_shock=0.5, x_int=0.7, nsteps=nsteps)
    ny, nx = case["rho"].shape
    print(f"[parity] shock_interface {nx}x{ny} fp64 {nsteps} steps (tile form)", flush=True)
    with lib.Solver(case["params"]) as s:
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(nsteps)
        s.sync()
        mg = s.macros()
    margin = 2 * nsteps + 2
    for x0, y0 in [(0, 100), (2030, 7), (2880, 4200 - 40), (4096 - 80, 3000)]:
        nxw, nyw = 80, 80
        p, sl = _window_case(case, x0, nxw, y0, nyw)
        fo = orc.run(p, sl(case["rho"]), sl(case["ux"]), sl(case["uy"]), sl(case["T"]), nsteps)
        mo = orc.macros(p, fo)
        xs = slice(0 if x0 == 0 else margin, nxw if x0 + nxw == nx else nxw - margin)
        ys = slice(margin, nyw - margin)
        assert_parity(tuple(sl(m)[ys, xs] for m in mg), tuple(m[ys, xs] for m in mo), TOL["fp64"], 1.4,
                      f"window x0={x0} y0={y0}")
