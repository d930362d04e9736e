"""Host-side check of the two-steps-per-launch schedule (k_march2).

The kernel's two wavefronts advance in lockstep, one barrier per iteration,
through H + 6 iterations for a band of H output rows; r(k) is the row at
march position k.  The first wavefront makes rows r(-2) .. r(1) at
iterations 0..3 and r(2) .. r(H + 1) at iterations 5..H + 4 into a ring of
four rows (row y in slot (y + 4) mod 4); the second loads r(-2) .. r(1) at
iteration 4 and, at iteration k + 6, reads r(k + 2) and makes output row
r(k).  Outflow ghost rows are read at the row they repeat.  This test
replays that schedule for every boundary pair, band position, direction and
band height on small grids and checks that every row read was written at an
earlier iteration and not overwritten since, and that no slot is read in the
iteration that writes it.
"""
import pytest

PER, EQ, OUT = 0, 1, 2
RING = 4


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
    written = {}
    for t in range(H + 6):
        if t == 4:
            reads = [r(k) for k in (-2, -1, 0, 1)]
        elif t >= 6:
            reads = [r(t - 6 + 2)]
        else:
            reads = []
        slots_read = set()
        for row in reads:
            s = source_out(row, ny, lo, hi)
            assert -2 <= s <= ny + 1
            slot = (s + 4) % RING
            assert slot in written and written[slot] == (s, written[slot][1]) and written[slot][1] < t, \
                (ny, lo, hi, yb, ye, d, t, row)
            slots_read.add(slot)
        kp = t - 2 if t <= 3 else (t - 3 if 5 <= t <= H + 4 else None)
        if kp is not None:
            row = r(kp)
            assert -2 <= row <= ny + 1
            slot = (row + 4) % RING
            assert slot not in slots_read, (ny, lo, hi, yb, ye, d, t, row)
            written[slot] = (row, t)
    # the second wavefront made every output row once
    return H


@pytest.mark.parametrize("lo,hi", [(PER, PER), (EQ, EQ), (OUT, OUT), (EQ, OUT), (OUT, EQ)])
def test_ring_reads_follow_writes(lo, hi):
    n = 0
    for ny in range(1, 14):
        for H in range(1, ny + 1):
            for yb in range(ny):
                ye = min(yb + H, ny)
                for d in (1, -1):
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
