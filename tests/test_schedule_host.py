"""CPU: the register-direct kernels' persistent tile schedules, restated from their
device arithmetic (WaveCursor for free waves, HalfCursor for the out-of-phase lockstep
groups of k_flux_rd.h), over many tile counts and grids: every tile is taken exactly
once, every wave of a workgroup runs the same number of lockstep rounds (each round has
one barrier per wave, so unequal counts would leave a barrier unmatched), and a wave
that holds a tile always sits in a round the workgroup runs; the same under any rotation
of a XCD's workgroup order, and for a batch the rotation handed from one interface to
the next (rd_next_rot) spreads the interfaces' partial last rounds over different
workgroups.  The GPU tests test_register_direct_schedule_any_grid and the batch tests
check the kernels themselves."""
import pytest

XCDS = 8


def xcd_workgroups(grid, blk):
    xcd = blk % XCDS
    return grid // XCDS + (1 if grid % XCDS > xcd else 0)


def place(grid, blk, rot):
    return (blk // XCDS + rot) % xcd_workgroups(grid, blk)


def next_rot(length, unit, grid, blk, rot):
    nwg = xcd_workgroups(grid, blk)
    e = ((max(length, 0) % (nwg * unit)) + unit - 1) // unit
    assert 0 <= e <= nwg
    return (rot - e + nwg) % nwg


def wave_cursor_next_rot(n, grid, waves, blk, rot):
    per = (n + XCDS - 1) // XCDS
    base = (blk % XCDS) * per
    return next_rot(min(n, base + per) - base, waves, grid, blk, rot)


def half_cursor_next_rot(n, grid, waves, blk, rot):
    per = (n + XCDS - 1) // XCDS
    base = min(n, (blk % XCDS) * per)
    lim = min(n, base + per)
    return next_rot((lim - base + 1) // 2, waves // 2, grid, blk, rot)


def wave_cursor(n, grid, waves, blk, wave, rot=0):
    xcd = blk % XCDS
    stride = xcd_workgroups(grid, blk) * waves
    per = (n + XCDS - 1) // XCDS
    base = xcd * per
    limit = min(n, base + per)
    k = base + place(grid, blk, rot) * waves + wave
    tiles, rounds = [], 0
    while k - wave < limit:            # round_valid: the workgroup's first wave has a tile
        if k < limit:
            tiles.append(k)
        k += stride
        rounds += 1
    return tiles, rounds


def half_cursor(n, grid, waves, blk, wave, rot=0):
    xcd = blk % XCDS
    nwg = xcd_workgroups(grid, blk)
    per = (n + XCDS - 1) // XCDS
    base = min(n, xcd * per)
    lim = min(n, base + per)
    mid = base + (lim - base + 1) // 2
    hw = waves // 2
    grp = 0 if wave < hw else 1
    stride = nwg * hw
    first = base + place(grid, blk, rot) * hw
    k = (mid if grp else base) + place(grid, blk, rot) * hw + (wave - grp * hw)
    limit = lim if grp else mid
    tiles, rounds = [], 0
    while first < mid:                 # round_valid: the first group's first wave has a tile
        if k < limit:
            tiles.append(k)
        k += stride
        first += stride
        rounds += 1
    assert k >= limit, "a tile left after the last round"
    return tiles, rounds


@pytest.mark.parametrize("cursor,waves", [(wave_cursor, 4), (wave_cursor, 8), (half_cursor, 8),
                                          (half_cursor, 4)])
@pytest.mark.parametrize("grid", [8, 9, 11, 13, 16, 24, 40, 64, 256, 520])
@pytest.mark.parametrize("rot", [0, 1, 5, 31])
def test_every_tile_once_and_equal_rounds(cursor, waves, grid, rot):
    for n in list(range(0, 90)) + [200, 1000, 3456, 17920, 22000, 30416]:
        taken = []
        for blk in range(grid):
            r_blk = rot % xcd_workgroups(grid, blk)      # a rotation is below the XCD's count
            per_wave = [cursor(n, grid, waves, blk, w, r_blk) for w in range(waves)]
            rounds = {r for _, r in per_wave}
            assert len(rounds) == 1, (n, grid, blk, rounds)
            for tiles, _ in per_wave:
                taken += tiles
        assert sorted(taken) == list(range(n)), (n, grid)


def batch_rounds(tile_counts, grid, waves, cursor, rotate):
    """Rounds each workgroup runs over a batch of interfaces taken one after the other,
    with the rotation handed on (rotate) or every interface in the same order."""
    nxt = half_cursor_next_rot if cursor is half_cursor else wave_cursor_next_rot
    totals = []
    taken = [[] for _ in tile_counts]
    for blk in range(grid):
        rot, total = 0, 0
        for i, n in enumerate(tile_counts):
            per_wave = [cursor(n, grid, waves, blk, w, rot) for w in range(waves)]
            rounds = {r for _, r in per_wave}
            assert len(rounds) == 1
            total += rounds.pop()
            for tiles, _ in per_wave:
                taken[i] += tiles
            if rotate:
                rot = nxt(n, grid, waves, blk, rot)
        totals.append(total)
    for i, n in enumerate(tile_counts):
        assert sorted(taken[i]) == list(range(n))
    return totals


def test_batch_rotation_turbine_like():
    # the turbine-like batch: N = 7 annulus 320x125 (22 tiles per row, 8 node rows),
    # N = 5 annulus 256x72 (18 x 6), N = 3 plane 64x32 (5 x 4); 256 eight-wave workgroups.
    # Per XCD and half: 1375 tiles = 10 rounds of 128 + 95 (24 workgroups), 486 = 3 x 128
    # + 102 (26), 40 (10): without the rotation workgroups 0-9 of every XCD run
    # 11 + 4 + 1 = 16 rounds, with it no workgroup runs more than 15.
    counts = [22 * 8 * 125, 18 * 6 * 72, 5 * 4 * 32]
    plain = batch_rounds(counts, 256, 8, half_cursor, rotate=False)
    rotated = batch_rounds(counts, 256, 8, half_cursor, rotate=True)
    assert max(plain) == 16 and max(rotated) == 15
    assert sum(plain) == sum(rotated)


@pytest.mark.parametrize("cursor,waves", [(half_cursor, 8), (wave_cursor, 4), (wave_cursor, 8)])
@pytest.mark.parametrize("grid", [8, 13, 40, 256])
def test_batch_rotation_never_longer(cursor, waves, grid):
    import random
    rng = random.Random(grid * 10 + waves)
    for _ in range(25):
        counts = [rng.choice([0, 1, 7, 64, 640, 3456, 7776, 22000]) for _ in range(rng.randint(1, 4))]
        plain = batch_rounds(counts, grid, waves, cursor, rotate=False)
        rotated = batch_rounds(counts, grid, waves, cursor, rotate=True)
        assert max(rotated) <= max(plain), (counts, grid)
        assert sum(rotated) == sum(plain)
