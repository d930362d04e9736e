"""Host-side check of the two-steps-per-launch schedule (k_march2).

The kernel's two wavefronts advance in lockstep, one barrier per iteration,
through H + 6 iterations for a band of H output rows; r(k) is the row at
march position k.  The first wavefront makes rows r(-2) .. r(1) at
iterations 0..3 and r(2) .. r(H + 1) at iterations 5..H + 4 into a ring of
four rows (row y in slot (y + 4) mod 4); the second reads r(-2) .. r(1) at
iteration 4 and, at iteration k + 6, reads r(k), r(k + 1) and r(k + 2) and
makes output row r(k) (it copies r(k + 2) into registers then, and in FP64
reads the neighbouring columns of r(k) again; the variant that reads every
row where it is used needs all three).  Outflow ghost rows are read at the
row they repeat.

Walls along y (bands walk up only): the rows the first step makes at a
wall's node row and ghost row are not valid; on the high side the first
wavefront refills its rows r(k) >= ny - 1 from row ny - 2 instead of
stepping them, at their own iterations; on the low side the second
wavefront refills rows 0 and -1 (those at or above r(-2)) from row 1 at
iteration 3.

This test replays that schedule for every boundary pair, band position,
direction and band height on small grids and checks that every row read
holds a valid value of that row written at an earlier iteration (or earlier
in the same iteration by the same wavefront) and not overwritten since, and
that no slot is touched by both wavefronts in one iteration when either
writes it.
"""
import pytest

PER, EQ, OUT, WALL = 0, 1, 2, 3
RING = 4
REFILL = True      # the wall refills (off only to check that the replay notices)


def source_out(c, n, lo, hi):
    if c < 0 and lo == OUT:
        return 0
    if c >= n and hi == OUT:
        return n - 1
    return c


def replay(ny, lo, hi, yb, ye, d):
    H = ye - yb
    j0 = yb if d > 0 else ye - 1
    r = lambda k: j0 + d * k
    slot_of = lambda row: (row + 4) % RING
    ring = {}                       # slot -> (row, valid)

    def valid_step(row):
        # a row the first step makes from the state at step n
        if lo == WALL and row <= 0:
            return False
        if hi == WALL and row >= ny - 1:
            return False
        return True

    lead = max(0, ye + 3 - ny) if (REFILL and d > 0 and hi == WALL) else 0
    nn = H + 4 - lead
    first = {}                      # iteration -> ops of the first wavefront
    for k in range(-2, H + 2):
        t = k + 2 if k <= 1 else k + 3
        row = r(k)
        assert -2 <= row <= ny + 1
        if k <= nn - 3:
            first[t] = [("w", row, valid_step(row))]
        else:
            assert hi == WALL and row >= ny - 1
            first[t] = [("r", ny - 2), ("w", row, True)]
    second = {}
    if REFILL and d > 0 and lo == WALL and yb <= 2:
        second[3] = [("r", 1)] + [("w", w, True) for w in (0, -1) if w >= yb - 2]
    second[4] = [("r", source_out(r(k), ny, lo, hi)) for k in (-2, -1, 0, 1)]
    for t in range(6, H + 6):
        second[t] = [("r", source_out(r(t - q), ny, lo, hi)) for q in (6, 5, 4)]

    for t in range(H + 6):
        touched = {}
        new = {}
        for wave, ops in ((0, first.get(t, [])), (1, second.get(t, []))):
            for op in ops:
                slot = slot_of(op[1])
                touched.setdefault(slot, set()).add((wave, op[0]))
                if op[0] == "r":
                    # own earlier writes in this iteration, else the ring as
                    # the previous barrier left it
                    have = new.get((wave, slot), ring.get(slot))
                    assert have == (op[1], True), (ny, lo, hi, yb, ye, d, t, wave, op, have)
                else:
                    new[(wave, slot)] = (op[1], op[2])
        for slot, who in touched.items():
            waves = {w for w, _ in who}
            writes = any(o == "w" for _, o in who)
            assert not (len(waves) == 2 and writes), (ny, lo, hi, yb, ye, d, t, slot, who)
        for (wave, slot), v in new.items():
            ring[slot] = v
    return H


def bands(ny, lo, hi):
    y0, y1 = (1 if lo == WALL else 0), (ny - 1 if hi == WALL else ny)
    dirs = (1,) if WALL in (lo, hi) else (1, -1)
    for H in range(1, y1 - y0 + 1):
        for yb in range(y0, y1):
            for d in dirs:
                yield yb, min(yb + H, y1), d


@pytest.mark.parametrize("lo,hi", [(PER, PER), (EQ, EQ), (OUT, OUT), (EQ, OUT), (OUT, EQ),
                                   (WALL, WALL), (WALL, OUT), (WALL, EQ), (OUT, WALL), (EQ, WALL)])
def test_ring_reads_follow_writes(lo, hi):
    n = 0
    for ny in range(1, 14):
        if ny < 1 + (lo == WALL) + (hi == WALL):
            continue
        for yb, ye, d in bands(ny, lo, hi):
            n += replay(ny, lo, hi, yb, ye, d)
    assert n > 0


def test_ring_of_three_would_not_do():
    # the ring needs four rows: with three, priming reads r(-2) .. r(1)
    # while the slot of r(-2) would be rewritten with r(1)
    global RING
    saved, RING = RING, 3
    try:
        with pytest.raises(AssertionError):
            replay(20, PER, PER, 5, 15, 1)
    finally:
        RING = saved


@pytest.mark.parametrize("lo,hi,yb,ye", [(WALL, OUT, 1, 5), (WALL, OUT, 2, 5), (OUT, WALL, 4, 11),
                                         (OUT, WALL, 4, 10), (OUT, WALL, 10, 11)])
def test_unrefilled_walls_are_caught(lo, hi, yb, ye):
    # without the refills the second step reads the first step's own values
    # at a wall's rows, which are not the wall's
    global REFILL
    saved, REFILL = REFILL, False
    try:
        with pytest.raises(AssertionError):
            replay(12, lo, hi, yb, ye, 1)
    finally:
        REFILL = saved
