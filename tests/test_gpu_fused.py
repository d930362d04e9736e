"""Two steps per launch against one step per launch, on the GPU.

The fused pair kernel takes step n -> n+1 into a ring of rows in LDS and
step n+1 -> n+2 from there; every node value is formed from the same
operands in the same order as in the one-step kernel, so the state must
agree to the last bit after any number of steps (odd counts end with one
single step).  Cases cover every boundary kind on each axis (periodic
ghosts computed by translation, equilibrium ghosts passed through, outflow
ghosts read at their source lane or row), grids narrower than a strip,
ragged strips, one-row and few-row grids (a band reaching both edges),
launches with many bands, both storage precisions and all four limiters.
Walls along y are refilled inside the pair (the wall rows of the first
step's result, written into the ring of rows); cases cover them with every
x boundary kind, one or both walls, and band layouts whose bands reach a
wall within one or two rows.  The march kernels also refill the walls of
their own output (along y), where the tile form launches a refill kernel;
all forms agree bitwise.  Walls along x are rejected for fusion.  The
fused path is also compared with the oracle directly (every boundary kind,
both precisions), and the other GPU tests run it wherever it is the default
(large grids, e.g. the full 4096 x 1024 shock-interface windows).
"""
import numpy as np
import pytest

from parity import TOL, assert_parity, f_rel
from paper_1305_4736_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_4736_amd import mrtfd
    return mrtfd


P, O = W.bc("periodic"), W.bc("outflow")
E1, E2 = W.bc("equilibrium", 1.1, 0.05, -0.02, 0.9), W.bc("equilibrium", 0.8, -0.1, 0.03, 1.2)
AXES = {"P": (P, P), "E": (E1, E2), "O": (O, O), "EO": (E1, O), "OE": (O, E2)}
WL, WH = W.bc("wall", 1.0, 0.0, 0.0, 1.0), W.bc("wall", 1.0, 0.15, 0.0, 1.05)
YWALLS = {"WW": (WL, WH), "WO": (WL, O), "WE": (WL, E2), "OW": (O, WH), "EW": (E1, WH)}


def state(lib, case, per_launch, nsteps):
    with lib.Solver(case["params"]) as s:
        s.steps_per_launch = per_launch
        assert s.steps_per_launch == per_launch
        s.init(case["rho"], case["ux"], case["uy"], case["T"])
        s.step(nsteps)
        s.sync()
        return s.get_f(), s.macros()


def check(lib, case, nsteps):
    print(f"[fused] {case['name']} {case['params']['precision']} {case['params']['limiter']} "
          f"bc={[b['kind'] for b in case['params']['bc']]} n={nsteps}", flush=True)
    f1, m1 = state(lib, case, 1, nsteps)
    f2, m2 = state(lib, case, 2, nsteps)
    assert np.all(np.isfinite(f1))
    bad = np.argwhere(f1 != f2)
    assert bad.size == 0, f"{len(bad)} values differ, first (plane, y, x) {bad[:4].tolist()}"
    for a, b in zip(m1, m2):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("xa", list(AXES))
@pytest.mark.parametrize("ya", list(AXES))
def test_every_boundary_pair(lib, xa, ya):
    bcs = list(AXES[xa]) + list(AXES[ya])
    c = W.random_smooth(131, 70, seed=7, bcs=bcs, jumps=True)
    check(lib, c, 9)


@pytest.mark.parametrize("nx,ny", [(1, 1), (3, 2), (5, 1), (7, 9), (56, 5), (57, 6), (60, 3), (113, 1),
                                   (400, 1), (1, 37), (2, 300)])
@pytest.mark.parametrize("axes", ["PP", "EO", "OP"])
def test_small_and_ragged_grids(lib, nx, ny, axes):
    bcs = list(AXES[axes[0]]) + list(AXES[axes[1]])
    c = W.random_smooth(nx, ny, seed=nx * 31 + ny, bcs=bcs, jumps=nx > 4)
    check(lib, c, 8)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("limiter", ["mc", "minmod", "lw", "upwind"])
def test_precisions_and_limiters(lib, precision, limiter):
    c = W.random_smooth(300, 97, seed=3, bcs=[E1, O, P, P], limiter=limiter, precision=precision, jumps=True)
    check(lib, c, 7)


def test_many_bands_and_long_run(lib):
    # 1500 x 700: ~27 strips, ~38 bands of ~18 rows walking in both directions
    c = W.random_smooth(1500, 700, seed=11, bcs=[E1, O, P, P], jumps=True)
    check(lib, c, 40)


def test_shock_interface_full_size(lib):
    c = W.shock_interface()
    check(lib, c, 6)


@pytest.mark.parametrize("xa", ["P", "E", "O"])
@pytest.mark.parametrize("yw", list(YWALLS))
def test_walls_along_y(lib, xa, yw):
    bcs = list(AXES[xa]) + list(YWALLS[yw])
    c = W.random_smooth(131, 70, seed=8, bcs=bcs, jumps=True)
    check(lib, c, 9)


# Band layouts (1024 resident pairs): one-row bands, where every band near
# a wall reaches it within one or two rows (3..7 rows); and taller bands
# whose last band has 1 row (1000 x 297: 6-row bands, the one before it
# ends two rows below the wall; 50 x 2001: 2-row bands), 2 rows
# (1000 x 298), 4 rows (1000 x 300) or 14 rows (1500 x 700).
@pytest.mark.parametrize("nx,ny", [(64, 3), (64, 4), (5, 5), (60, 6), (57, 7), (1000, 297), (1000, 298),
                                   (1000, 300), (50, 2001), (1500, 700)])
@pytest.mark.parametrize("xa", ["P", "E"])
def test_wall_band_layouts(lib, nx, ny, xa):
    bcs = list(AXES[xa]) + [WL, WH]
    c = W.random_smooth(nx, ny, seed=nx + ny, bcs=bcs, jumps=nx > 4)
    check(lib, c, 8)


@pytest.mark.parametrize("limiter", ["mc", "minmod"])
def test_walls_fp32(lib, limiter):
    c = W.random_smooth(1000, 297, seed=9, bcs=[E1, O, WL, WH], limiter=limiter, precision="fp32", jumps=True)
    check(lib, c, 7)


def test_couette_fused(lib):
    c = W.couette(pr=1.0, nx=130, ny=200)
    check(lib, c, 50)


def test_random_configurations(lib):
    # a seeded sweep over grid sizes (1 to 300 columns, ragged strips), every
    # boundary pair with walls along y, both precisions, all limiters and odd
    # and even step counts
    rng = np.random.default_rng(20260)
    xkinds = ["P", "E", "O", "EO", "OE"]
    ykinds = xkinds + list(YWALLS)
    limiters = ["mc", "minmod", "lw", "upwind"]
    for k in range(100):
        nx = int(round(np.exp(rng.uniform(0.0, np.log(300)))))
        ya = ykinds[rng.integers(len(ykinds))]
        ny = int(rng.integers(3 if ya in YWALLS else 1, 120))
        xa = xkinds[rng.integers(len(xkinds))]
        bcs = list(AXES[xa]) + list(YWALLS[ya] if ya in YWALLS else AXES[ya])
        c = W.random_smooth(nx, ny, seed=1000 + k, bcs=bcs, limiter=limiters[rng.integers(4)],
                            precision=["fp64", "fp32"][rng.integers(2)], jumps=nx > 4)
        check(lib, c, int(rng.integers(1, 12)))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wall_refill_forms_agree(lib, precision):
    # walls along y are refilled by the march kernels themselves (one or two
    # steps per launch, batched strips); the tile form and walls along x keep
    # the refill launch: all give the same bits
    cases = [W.random_smooth(131, 70, seed=31, bcs=[P, P, WL, WH], precision=precision, jumps=True),
             W.random_smooth(90, 41, seed=32, bcs=[E1, O, WL, O], precision=precision, jumps=True),
             W.random_smooth(77, 35, seed=33, bcs=[O, O, E1, WH], precision=precision, jumps=True),
             W.couette(pr=1.0, nx=64, ny=50, precision=precision),
             W.random_smooth(60, 40, seed=34, bcs=[WL, WH, P, P], precision=precision, jumps=True)]
    n = 9
    for c in cases:
        xwalls = c["params"]["bc"][0]["kind"] == "wall"
        print(f"[refill-forms] {c['name']} {precision} x walls {xwalls}", flush=True)
        ref, _ = state(lib, c, 1, n)
        assert np.all(np.isfinite(ref))
        got = {} if xwalls else {"two steps per launch": state(lib, c, 2, n)[0]}
        for shape in ("strips", "tile32x8", "tile64x4"):
            with lib.Batch(2, precision=precision) as b:
                slot = b.add(c["params"], c["rho"], c["ux"], c["uy"], c["T"], nsteps=n)
                b.set_shape(slot, shape)
                b.step(n)
                got["batch " + shape] = b.get_f(slot)
        for form, f in got.items():
            assert np.array_equal(ref, f), (c["name"], form)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_walls_hold_a_matching_uniform_state(lib, axis):
    # as in the oracle's invariants: a uniform equilibrium moving along NEE
    # walls at their speed and temperature stays put (walls along y in both
    # launch forms; along x one step per launch)
    if axis == "y":
        w = W.bc("wall", 1.0, 0.1, 0.0, 0.9)
        bcs, state = [P, P, w, w], (1.3, 0.1, 0.0, 0.9)
    else:
        w = W.bc("wall", 1.0, 0.0, -0.08, 0.9)
        bcs, state = [w, w, P, P], (1.3, 0.0, -0.08, 0.9)
    c = W.random_smooth(300, 200, seed=4, bcs=bcs)
    shp = (c["params"]["ny"], c["params"]["nx"])
    for per_launch in ((1, 2) if axis == "y" else (1,)):
        with lib.Solver(c["params"]) as s:
            s.steps_per_launch = per_launch
            s.init(*[np.full(shp, v) for v in state])
            f0 = s.get_f()
            s.step(30)
            s.sync()
            f1 = s.get_f()
        assert np.abs(f1 - f0).max() <= 1e-13 * np.abs(f0).max(), (axis, per_launch)


def test_fusion_rules(lib):
    c = W.random_smooth(64, 40, bcs=[WL, WH, P, P])
    with lib.Solver(c["params"]) as s:
        assert s.steps_per_launch == 1          # walls along x: never fused
        with pytest.raises(lib.MRTFDError):
            s.steps_per_launch = 2
        with pytest.raises(lib.MRTFDError):
            s.steps_per_launch = 3
        assert s.steps_per_launch == 1
    c = W.random_smooth(64, 40, bcs=[P, P, WL, WH])
    with lib.Solver(c["params"]) as s:
        assert s.steps_per_launch == 1          # walls along y: fused on request
        s.steps_per_launch = 2
        assert s.steps_per_launch == 2
    c = W.random_smooth(1024, 512, bcs=[P, P, WL, WH])
    with lib.Solver(c["params"]) as s:
        assert s.steps_per_launch == 2          # and by default on a large grid
    c = W.random_smooth(1024, 512)
    with lib.Solver(c["params"]) as s:
        assert s.steps_per_launch == 2          # FP64 on a large grid: fused by default
        with pytest.raises(lib.MRTFDError):
            s.steps_per_launch = 0
    c = W.random_smooth(64, 40)
    with lib.Solver(c["params"]) as s:
        assert s.steps_per_launch == 1          # small grid: one step per launch by default
        s.steps_per_launch = 2
        assert s.steps_per_launch == 2
    c = W.random_smooth(1024, 256, precision="fp32")
    with lib.Solver(c["params"]) as s:
        assert s.steps_per_launch == 1          # FP32 fuses from somewhat taller bands than FP64
    c = W.random_smooth(1024, 512, precision="fp32")
    with lib.Solver(c["params"]) as s:
        assert s.steps_per_launch == 2


@pytest.mark.parametrize("axes", ["PP", "EO", "OE", "EP", "OO", "P-WW", "E-WO", "O-EW"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_against_oracle(lib, orc, axes, precision):
    if "-" in axes:
        xa, yw = axes.split("-")
        bcs = list(AXES[xa]) + list(YWALLS[yw])
    else:
        bcs = list(AXES[axes[0]]) + list(AXES[axes[1]])
    c = W.random_smooth(150, 61, seed=5, bcs=bcs, precision=precision, jumps=True)
    n = 10
    print(f"[fused-oracle] 150x61 {axes} {precision} n={n}", flush=True)
    with lib.Solver(c["params"]) as s:
        s.steps_per_launch = 2
        s.init(c["rho"], c["ux"], c["uy"], c["T"])
        s.step(n)
        s.sync()
        mg, fg = s.macros(), s.get_f()
    p = c["params"]
    fo = orc.run(p, c["rho"], c["ux"], c["uy"], c["T"], n)
    assert_parity(mg, orc.macros(p, fo), TOL[precision], 1.4, f"fused {axes} {precision}")
    if precision == "fp64":
        assert f_rel(fg, fo) <= TOL["fp64"]


@pytest.mark.parametrize("node", [(0, 0), (4, 55), (17, 56), (40, 111), (69, 149)])
@pytest.mark.parametrize("nsteps", [1, 2, 5])
def test_nonfinite_is_reported_fused(lib, node, nsteps):
    # nodes at the grid's corners and on strip edges (56-column strips)
    c = W.random_smooth(150, 70, seed=4, bcs=[E1, O, P, P])
    with lib.Solver(c["params"]) as s:
        s.steps_per_launch = 2
        s.init(c["rho"], c["ux"], c["uy"], c["T"])
        s.step(2)
        s.sync()
        f = s.get_f()
        f[:, node[0], node[1]] = np.nan
        s.set_f(f)
        s.step(nsteps)
        with pytest.raises(lib.NonFiniteError):
            s.sync()
        s.sync()    # the flag was cleared
