"""CPU: the register-direct kernels' persistent tile schedules, restated from their
device arithmetic (WaveCursor for free waves, HalfCursor for the out-of-phase lockstep
groups of k_flux_rd.h), over many tile counts and grids: every tile is taken exactly
once, every wave of a workgroup runs the same number of lockstep rounds (each round has
one barrier per wave, so unequal counts would leave a barrier unmatched), and a wave
that holds a tile always sits in a round the workgroup runs.  The GPU test
test_register_direct_schedule_any_grid checks the kernels themselves on such grids."""
import pytest

XCDS = 8


def wave_cursor(n, grid, waves, blk, wave):
    xcd = blk % XCDS
    stride = (grid // XCDS + (1 if grid % XCDS > xcd else 0)) * waves
    per = (n + XCDS - 1) // XCDS
    base = xcd * per
    limit = min(n, base + per)
    k = base + (blk // XCDS) * waves + wave
    tiles, rounds = [], 0
    while k - wave < limit:            # round_valid: the workgroup's first wave has a tile
        if k < limit:
            tiles.append(k)
        k += stride
        rounds += 1
    return tiles, rounds


def half_cursor(n, grid, waves, blk, wave):
    xcd = blk % XCDS
    nwg = grid // XCDS + (1 if grid % XCDS > xcd else 0)
    per = (n + XCDS - 1) // XCDS
    base = min(n, xcd * per)
    lim = min(n, base + per)
    mid = base + (lim - base + 1) // 2
    hw = waves // 2
    grp = 0 if wave < hw else 1
    stride = nwg * hw
    first = base + (blk // XCDS) * hw
    k = (mid if grp else base) + (blk // XCDS) * hw + (wave - grp * hw)
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
def test_every_tile_once_and_equal_rounds(cursor, waves, grid):
    for n in list(range(0, 90)) + [200, 1000, 3456, 17920, 22000, 30416]:
        taken = []
        for blk in range(grid):
            per_wave = [cursor(n, grid, waves, blk, w) for w in range(waves)]
            rounds = {r for _, r in per_wave}
            assert len(rounds) == 1, (n, grid, blk, rounds)
            for tiles, _ in per_wave:
                taken += tiles
        assert sorted(taken) == list(range(n)), (n, grid)
