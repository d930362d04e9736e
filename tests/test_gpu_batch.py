"""GPU tests of the batched form: many instances of different sizes, states,
rates and boundaries advance in shared persistent launches.

* each slot matches the FP64 oracle (1e-11 FP64 storage, 2e-5 FP32);
* each slot's result is the same alone and in the mix (bitwise), and the
  same as the single-instance entry point;
* every shape class (LDS tiles and row-marching strips) gives the same
  bits as the single-instance entry point, also when a slot changes class
  mid-run;
* per-slot step budgets, slots added and removed mid-run, the autotuner's
  shape reassignment and a non-finite slot leave the other slots' results
  unchanged.
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
    from paper_1305_4736_amd import mrtfd
    return mrtfd


P, E, O = W.bc("periodic"), W.bc("equilibrium", 1.1, 0.05, -0.02, 0.9), W.bc("outflow")
WL, WH = W.bc("wall", 1.0, 0.0, 0.0, 1.0), W.bc("wall", 1.0, 0.15, 0.0, 1.05)


def mixed_cases(limiter="mc"):
    cs = [
        W.riemann_1d((1.0, 0.1, 1.0), (0.3, 0.0, 0.4), 1.4, 300, ny=1, limiter=limiter, nsteps=0),
        W.random_smooth(67, 13, seed=1, bcs=[P, P, P, P], limiter=limiter, jumps=True),
        W.random_smooth(50, 20, seed=2, bcs=[E, O, P, P], limiter=limiter, jumps=True),
        W.couette(pr=1.0, nx=4, ny=30, limiter=limiter),
        W.random_smooth(1, 37, seed=3, bcs=[P, P, P, P], limiter=limiter),
        W.riemann_1d((1.0, 0.0, 1.0), (0.5, 0.2, 0.5), 1.67, 200, ny=5, limiter=limiter, nsteps=0),
        W.random_smooth(130, 70, seed=4, bcs=[O, O, O, O], limiter=limiter, jumps=True),
        W.riemann_1d((2.0, 0.0, 2.0), (1.0, 0.0, 1.0), 1.2, 777, ny=1, limiter=limiter, nsteps=0),
    ]
    return cs


def add_all(batch, cases, budgets=None):
    slots = []
    for k, c in enumerate(cases):
        n = -1 if budgets is None else budgets[k]
        slots.append(batch.add(c["params"], c["rho"], c["ux"], c["uy"], c["T"], nsteps=n))
    return slots


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_oracle(lib, orc, precision):
    cases = mixed_cases()
    n = 40
    with lib.Batch(len(cases) + 3, precision=precision) as b:
        slots = add_all(b, cases)
        for s in slots:
            tx, ty = b.shape(s)
            assert (tx, ty) in {(32, 8), (64, 4), (128, 2), (256, 1)} or (tx == 60 and 1 <= ty <= 32)
        b.step(n)
        b.status()
        for c, s in zip(cases, slots):
            mg = b.macros(s)
            fo = orc.run(c["params"], c["rho"], c["ux"], c["uy"], c["T"], n)
            mo = orc.macros(c["params"], fo)
            gamma = (c["params"]["b"] + 2.0) / c["params"]["b"]
            assert_parity(mg, mo, TOL[precision], gamma, f"slot {s} {c['name']}")
            assert b.steps_done(s) == n


def test_alone_equals_mix(lib):
    cases = mixed_cases()
    n = 30
    with lib.Batch(len(cases)) as mix:
        slots = add_all(mix, cases)
        mix.step(n)
        in_mix = [mix.get_f(s) for s in slots]
    for c, fm in zip(cases, in_mix):
        with lib.Batch(1) as alone:
            s = alone.add(c["params"], c["rho"], c["ux"], c["uy"], c["T"])
            alone.step(n)
            assert np.array_equal(alone.get_f(s), fm), c["name"]
        with lib.Solver(c["params"]) as single:
            single.init(c["rho"], c["ux"], c["uy"], c["T"])
            single.step(n)
            assert np.array_equal(single.get_f(), fm), c["name"]


def single_f(lib, c, n):
    with lib.Solver(c["params"]) as single:
        single.init(c["rho"], c["ux"], c["uy"], c["T"])
        single.step(n)
        return single.get_f()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_shape_class_matches_single(lib, precision):
    cases = [dict(c, params=dict(c["params"], precision=precision)) for c in mixed_cases()]
    n = 17
    ref = [single_f(lib, c, n) for c in cases]
    for name, cls in lib.SHAPE_CLASSES.items():
        with lib.Batch(len(cases), precision=precision) as b:
            slots = add_all(b, cases)
            forced = []
            for k, s in enumerate(slots):
                try:
                    b.set_shape(s, cls)
                    forced.append(k)
                except lib.MRTFDError:
                    assert name == "row256" and cases[k]["params"]["ny"] > 1
            assert forced, name
            b.step(n)
            for k in forced:
                assert np.array_equal(b.get_f(slots[k]), ref[k]), (name, cases[k]["name"])


def test_class_change_mid_run(lib):
    # strips (which leave periodic / outflow ghosts stale) -> tile -> strips
    cases = mixed_cases()
    ref = [single_f(lib, c, 24) for c in cases]
    with lib.Batch(len(cases)) as b:
        slots = add_all(b, cases)
        for s in slots:
            b.set_shape(s, "strips")
        b.step(8)
        for s in slots:
            b.set_shape(s, "tile64x4")
        b.step(8)
        for s in slots:
            b.set_shape(s, "strips")
        b.step(8)
        for k, s in enumerate(slots):
            assert np.array_equal(b.get_f(s), ref[k]), cases[k]["name"]


def test_budgets_and_membership_changes(lib):
    cases = mixed_cases()
    budgets = [10, 25, -1, 5, 30, 0, 17, 12]
    with lib.Batch(len(cases) + 2) as b:
        slots = add_all(b, cases, budgets)
        b.step(10)
        # slot 0 has finished: remove it; a new instance joins with budget 20
        b.remove(slots[0])
        extra = W.random_smooth(45, 9, seed=9, bcs=[E, O, P, P], jumps=True)
        s_new = b.add(extra["params"], extra["rho"], extra["ux"], extra["uy"], extra["T"], nsteps=20)
        b.step(20)
        done = {s: b.steps_done(s) for s in slots[1:]}
        assert done[slots[1]] == 25 and done[slots[2]] == 30 and done[slots[3]] == 5
        assert done[slots[4]] == 30 and done[slots[5]] == 0 and done[slots[6]] == 17
        assert b.steps_done(s_new) == 20 and b.remaining(s_new) == 0 and b.remaining(slots[2]) == -1
        for k in range(1, len(cases)):
            c = cases[k]
            with lib.Solver(c["params"]) as single:
                single.init(c["rho"], c["ux"], c["uy"], c["T"])
                single.step(done[slots[k]])
                assert np.array_equal(single.get_f(), b.get_f(slots[k])), c["name"]
        with lib.Solver(extra["params"]) as single:
            single.init(extra["rho"], extra["ux"], extra["uy"], extra["T"])
            single.step(20)
            assert np.array_equal(single.get_f(), b.get_f(s_new))
        # a new budget continues from the current state
        b.set_steps(slots[1], 3)
        b.step(5)
        assert b.steps_done(slots[1]) == 3


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_step_rounds_match_one_step(lib, precision):
    # slots that take two steps per launch (strips, no walls along x, >= 8
    # rows) next to ones that cannot (short, tiles); odd and even budgets,
    # a restart and a class change mid-run, a slot joining late; the
    # 4096 x 1024 instance makes the two-step work fill the device twice
    # over, which two-step rounds need (it is compared by its macros).
    # Walls along y (refilled inside the pairs) with 32-row pair bands: the
    # last band 1 row (the one before it ending two rows below the wall),
    # 2 rows, a low wall only, a high wall only
    cases = mixed_cases() + [W.random_smooth(300, 150, seed=21, bcs=[E, O, P, P], jumps=True),
                             W.random_smooth(90, 64, seed=22, bcs=[O, O, O, O], jumps=True),
                             W.random_smooth(4096, 1024, seed=24, bcs=[E, O, P, P], jumps=True),
                             W.random_smooth(200, 35, seed=25, bcs=[P, P, WL, WH], jumps=True),
                             W.random_smooth(150, 36, seed=26, bcs=[E, O, WL, WH], jumps=True),
                             W.random_smooth(100, 67, seed=27, bcs=[O, O, WL, O], jumps=True),
                             W.random_smooth(90, 40, seed=28, bcs=[E, E, E, WH], jumps=True)]
    cases = [dict(c, params=dict(c["params"], precision=precision)) for c in cases]
    budgets = [7, 40, 33, -1, 40, 0, 21, 40, 39, 40, -1, 40, 31, -1, 38]
    late = W.random_smooth(120, 48, seed=23, bcs=[P, P, P, P], jumps=True)
    late = dict(late, params=dict(late["params"], precision=precision))
    out = {}
    for k in (1, 2):
        with lib.Batch(len(cases) + 1, precision=precision) as b:
            assert b.steps_per_launch == 2
            with pytest.raises(lib.MRTFDError):
                b.steps_per_launch = 3
            b.steps_per_launch = k
            assert b.steps_per_launch == k
            slots = add_all(b, cases, budgets)
            b.step(11)
            b.set_steps(slots[3], 9)
            b.set_shape(slots[7], "tile32x8")
            s_late = b.add(late["params"], late["rho"], late["ux"], late["uy"], late["T"], nsteps=25)
            b.step(13)
            b.set_shape(slots[7], "strips")
            b.step(20)
            out[k] = ([b.macros(s) if s == slots[10] else b.get_f(s) for s in slots + [s_late]],
                      [b.steps_done(s) for s in slots + [s_late]])
            one, two = b.rounds()
            assert (two > 0) if k == 2 else (two == 0), (k, one, two)
            assert one + 2 * two == 44
    assert out[1][1] == out[2][1]
    assert out[2][1] == [7, 40, 33, 9, 40, 0, 21, 40, 39, 40, 44, 40, 31, 44, 38, 25]
    for a, c, case in zip(out[1][0], out[2][0], cases + [late]):
        if isinstance(a, tuple):
            assert all(np.array_equal(x, y) for x, y in zip(a, c)), case["name"]
        else:
            assert np.array_equal(a, c), case["name"]
    # and against one instance alone
    for idx in (8, 9, 11, 12, 13, 14):
        c = cases[idx]
        with lib.Solver(c["params"]) as single:
            single.steps_per_launch = 1
            single.init(c["rho"], c["ux"], c["uy"], c["T"])
            single.step(out[2][1][idx])
            assert np.array_equal(single.get_f(), out[2][0][idx]), c["name"]


def test_autotune_keeps_results(lib):
    cases = mixed_cases()
    n = 12
    with lib.Batch(len(cases)) as b1:
        s1 = add_all(b1, cases)
        b1.step(n)
        ref = [b1.get_f(s) for s in s1]
    with lib.Batch(len(cases)) as b2:
        s2 = add_all(b2, cases)
        costs = b2.autotune()
        assert np.all(costs > 0) and np.all(np.isfinite(costs))
        b2.step(n)
        for r, s in zip(ref, s2):
            assert np.array_equal(r, b2.get_f(s))


def test_nonfinite_slot_is_isolated(lib):
    cases = mixed_cases()[:4]
    n = 8
    with lib.Batch(4) as clean:
        sc = add_all(clean, cases)
        clean.step(n)
        ref = [clean.get_f(s) for s in sc]
    with lib.Batch(4) as b:
        sb = add_all(b, cases)
        f = b.get_f(sb[1])
        f[:, 3, 10] = np.nan
        b.set_f(sb[1], f)
        b.step(n)
        with pytest.raises(lib.NonFiniteError) as e:
            b.status()
        assert list(np.nonzero(e.value.flags)[0]) == [sb[1]]
        for k in (0, 2, 3):
            assert np.array_equal(ref[k], b.get_f(sb[k]))
        b.status()      # cleared


def test_riemann_batch_subset_matches_oracle(lib, orc):
    # 16 instances of the seeded 512-instance batch, evenly spread over the
    # sizes of those with at most 20000 nodes (so the oracle finishes in
    # seconds), FP32 storage, autotuned classes, 40 steps
    cases, _ = W.riemann_batch(n=512, precision="fp32")
    small = sorted((c for c in cases if c["params"]["nx"] * c["params"]["ny"] <= 20000),
                   key=lambda c: c["params"]["nx"] * c["params"]["ny"])
    cases = [small[round(i * (len(small) - 1) / 15)] for i in range(16)]
    n = 40
    with lib.Batch(len(cases), precision="fp32") as b:
        slots = add_all(b, cases)
        b.autotune()
        b.step(n)
        b.status()
        for c, s in zip(cases, slots):
            p64 = dict(c["params"], precision="fp64")
            fo = orc.run(p64, c["rho"], c["ux"], c["uy"], c["T"], n)
            mo = orc.macros(p64, fo)
            gamma = (c["params"]["b"] + 2.0) / c["params"]["b"]
            assert_parity(b.macros(s), mo, TOL["fp32"], gamma, f"{c['name']} {c['params']['nx']}x{c['params']['ny']}")


def test_random_batch_matches_instances_alone(lib):
    # random instances (walls along y among them) with random budgets, odd
    # and even, stepped in uneven calls, a restart on the way; a 4096 x 1024
    # instance (2368 pair items of 32 rows x 56 columns) keeps the pair work
    # above the device's 1024 resident pairs, so two-step rounds run, and
    # slots with one step left step inside them.
    # Every slot ends bitwise equal to its instance run alone, one step per
    # launch.
    rng = np.random.default_rng(777)
    kinds = [[P, P, P, P], [E, O, P, P], [O, O, O, O], [P, P, WL, WH], [E, O, WL, O], [O, E, E, WH]]
    cases, budgets = [], []
    for k in range(24):
        nx = int(rng.integers(20, 600))
        ny = int(rng.integers(3, 90))
        c = W.random_smooth(nx, ny, seed=500 + k, bcs=kinds[rng.integers(len(kinds))], jumps=True,
                            precision="fp32")
        cases.append(c)
        budgets.append(int(rng.integers(0, 45)))
    cases.append(W.random_smooth(4096, 1024, seed=499, bcs=[E, O, P, P], jumps=True, precision="fp32"))
    budgets.append(-1)
    restart = 5
    with lib.Batch(len(cases), precision="fp32") as b:
        slots = add_all(b, cases, budgets)
        for n in (3, 10, 1, 7):
            b.step(n)
        b.set_steps(slots[restart], 9)       # 21 steps so far, then 9 more
        for n in (2, 13, 5, 6):
            b.step(n)
        got = [b.get_f(s) for s in slots[:-1]]
        done = [b.steps_done(s) for s in slots[:-1]]
        one, two = b.rounds()
        assert two > 0 and one + 2 * two == 47, (one, two)
    for k, c in enumerate(cases[:-1]):
        n_expect = min(budgets[k], 21) + 9 if k == restart else min(budgets[k], 47)
        assert done[k] == (9 if k == restart else n_expect), (k, done[k])
        with lib.Solver(c["params"]) as single:
            single.steps_per_launch = 1
            single.init(c["rho"], c["ux"], c["uy"], c["T"])
            single.step(n_expect)
            assert np.array_equal(single.get_f(), got[k]), (k, c["name"], c["params"]["bc"])


def test_full_riemann_batch_as_benchmarked(lib, orc):
    # the whole seeded 512-instance batch (28.5 M nodes) built and autotuned
    # as the benchmark builds it, 13 steps (two-step rounds and a last
    # one-step launch); twelve instances spread over all sizes, the largest
    # included, end bitwise equal to their instance run alone one step per
    # launch, and the three smallest of them match the oracle
    cases, _ = W.riemann_batch(n=512, precision="fp32")
    n = 13
    with lib.Batch(len(cases), precision="fp32", limiter="mc") as b:
        slots = add_all(b, cases)
        b.autotune()
        b.step(n)
        b.status()
        one, two = b.rounds()
        order = sorted(range(len(cases)), key=lambda k: cases[k]["params"]["nx"] * cases[k]["params"]["ny"])
        pick = [order[round(i * (len(order) - 1) / 11)] for i in range(12)]
        got = {k: b.get_f(slots[k]) for k in pick}
        mac = {k: b.macros(slots[k]) for k in pick[:3]}
    assert two > 0 and one + 2 * two == n, (one, two)
    for k in pick:
        c = cases[k]
        with lib.Solver(c["params"]) as single:
            single.steps_per_launch = 1
            single.init(c["rho"], c["ux"], c["uy"], c["T"])
            single.step(n)
            assert np.array_equal(single.get_f(), got[k]), (k, c["params"]["nx"], c["params"]["ny"])
    for k in pick[:3]:
        c = cases[k]
        p64 = dict(c["params"], precision="fp64")
        mo = orc.macros(p64, orc.run(p64, c["rho"], c["ux"], c["uy"], c["T"], n))
        gamma = (c["params"]["b"] + 2.0) / c["params"]["b"]
        assert_parity(mac[k], mo, TOL["fp32"], gamma, f"{c['name']} {c['params']['nx']}x{c['params']['ny']}")


def test_fitted_pair_bands_match_alone(lib):
    # Seven 4096 x 1024 instances give the two-step launches enough items
    # for the fitted band height to grow to 48 rows (1628 items each at
    # 48 rows, 1184 at 64, against eight per resident pair and 1.25 times
    # that to grow); slots with walls along y whose last 48-row band is 1,
    # 2 and 47 rows tall, next to the wall or not, and a ragged periodic
    # one take their bands in the balanced order beside them.  Every such
    # slot ends bitwise equal to its run alone, one step per launch.
    big = [W.random_smooth(4096, 1024, seed=600 + k, bcs=[E, O, P, P], jumps=True, precision="fp32")
           for k in range(7)]
    small = [W.random_smooth(130, 49, seed=610, bcs=[P, P, WL, WH], jumps=True, precision="fp32"),
             W.random_smooth(70, 50, seed=611, bcs=[E, O, WL, O], jumps=True, precision="fp32"),
             W.random_smooth(200, 95, seed=612, bcs=[O, O, O, WH], jumps=True, precision="fp32"),
             W.random_smooth(333, 97, seed=613, bcs=[P, P, P, P], jumps=True, precision="fp32")]
    n = 6
    print("[batch] fitted pair bands: 7 x 4096 x 1024 and 4 small slots, 6 steps", flush=True)
    with lib.Batch(len(big) + len(small), precision="fp32") as b:
        slots = add_all(b, big + small)
        b.step(n)
        b.status()
        rows = b.pair_rows()
        one, two = b.rounds()
        got = [b.get_f(s) for s in slots[len(big):]]
        big0 = b.macros(slots[0])
    assert rows == 48 and two == n // 2, (rows, one, two)
    for c, g in zip(small, got):
        with lib.Solver(c["params"]) as single:
            single.steps_per_launch = 1
            single.init(c["rho"], c["ux"], c["uy"], c["T"])
            single.step(n)
            assert np.array_equal(single.get_f(), g), c["name"]
    c = big[0]
    with lib.Solver(c["params"]) as single:
        single.steps_per_launch = 1
        single.init(c["rho"], c["ux"], c["uy"], c["T"])
        single.step(n)
        single.sync()
        alone = single.macros()
    assert all(np.array_equal(a, m) for a, m in zip(alone, big0))
