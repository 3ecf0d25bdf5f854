"""Pins of the oracle's loop, collapse and schedule definitions (CPU only).

The owner maps are checked against brute force that reaches the same
ownership by a different route (dealing iterations or chunks out one at a
time), and against invariants: every iteration owned exactly once, blocks
contiguous and ordered, block sizes differing by at most one.
"""
import itertools

import numpy as np
import pytest

from oracle import loops

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.mark.parametrize("lb,ub,step,expect", [
    (0, 10, 1, 10), (0, 10, 3, 4), (0, 9, 3, 3), (5, 5, 1, 0), (7, 3, 1, 0),
    (10, 0, -1, 10), (10, 0, -3, 4), (10, 1, -3, 3), (-4, 4, 2, 4), (3, 100, 7, 14),
])
def test_trip_count_closed_form(lb, ub, step, expect):
    assert loops.trip_count(lb, ub, step) == expect
    # brute force: count the iterations a C for-loop would run
    i, c = lb, 0
    while (i < ub if step > 0 else i > ub):
        c += 1
        i += step
    assert c == expect


def test_trip_count_rejects_zero_step():
    with pytest.raises(ValueError):
        loops.trip_count(0, 4, 0)


@pytest.mark.parametrize("dims", [
    [(0, 5, 1)],
    [(0, 3, 1), (0, 4, 1)],
    [(2, 11, 3), (-5, 5, 2)],
    [(9, 0, -2), (1, 7, 1), (4, -4, -3)],
    [(0, 1, 1), (0, 1, 1), (0, 6, 1)],
])
def test_collapse_decode_matches_nested_loops(dims):
    ref = loops.serial_iterations(dims)
    n = int(np.prod([loops.trip_count(*d) for d in dims]))
    assert len(ref) == n
    assert [loops.collapse_decode(dims, k) for k in range(n)] == ref


def _deal_blocks(n, P):
    """Near-equal block sizes by dealing items one by one, then prefix sums."""
    sizes = [0] * P
    for i in range(n):
        sizes[i % P] += 1
    starts = [0]
    for s in sizes:
        starts.append(starts[-1] + s)
    return [(starts[p], starts[p + 1]) for p in range(P)]


def _brute_static(n, T, U):
    team = [None] * n
    unit = [None] * n
    for t, (tlo, thi) in enumerate(_deal_blocks(n, T)):
        for u, (ulo, uhi) in enumerate(_deal_blocks(thi - tlo, U)):
            for k in range(tlo + ulo, tlo + uhi):
                team[k], unit[k] = t, u
    return team, unit


def _brute_chunk(n, T, U, c):
    team = [None] * n
    unit = [None] * n
    who = 0
    for lo in range(0, n, c):
        for k in range(lo, min(lo + c, n)):
            team[k], unit[k] = who // U, who % U
        who = (who + 1) % (T * U)
    return team, unit


def test_owner_static_brute_force_sweep():
    for n in list(range(0, 40)) + [63, 64, 65, 127, 300]:
        for T in (1, 2, 3, 5, 9):
            for U in (1, 2, 7, 64, 130):
                team, unit = loops.owner_map(n, T, U, loops.STATIC)
                bt, bu = _brute_static(n, T, U)
                assert team.tolist() == bt and unit.tolist() == bu, (n, T, U)


def test_owner_chunk_brute_force_sweep():
    for n in (0, 1, 17, 64, 100, 299, 300):
        for T in (1, 3, 9):
            for U in (1, 4, 64, 130):
                for c in (1, 2, 4, 17):
                    team, unit = loops.owner_map(n, T, U, loops.STATIC_CHUNK, c)
                    bt, bu = _brute_chunk(n, T, U, c)
                    assert team.tolist() == bt and unit.tolist() == bu, (n, T, U, c)


@pytest.mark.parametrize("n,T,U", [(1000, 7, 13), (4099, 16, 64), (5, 8, 8)])
def test_owner_static_invariants(n, T, U):
    team, unit = loops.owner_map(n, T, U)
    flat = team * U + unit
    assert (flat >= 0).all()
    # contiguous and ordered: flat id never decreases along k
    assert (np.diff(flat) >= 0).all()
    counts = np.bincount(flat, minlength=T * U)
    # team sizes differ by at most one, larger teams first
    tsz = np.bincount(team, minlength=T)
    assert tsz.max() - tsz.min() <= 1 and (np.diff(tsz) <= 0).all()
    assert counts.sum() == n


def test_owner_distribute_variants():
    n, T, U = 103, 5, 4
    team, unit = loops.owner_map(n, T, U, loops.STATIC, 0, loops.TEAMS)
    assert (unit == 0).all()
    assert [int((team == t).sum()) for t in range(T)] == [21, 21, 21, 20, 20]
    team, unit = loops.owner_map(n, 1, U, loops.STATIC, 0, loops.UNITS)
    assert (team == 0).all() and [int((unit == u).sum()) for u in range(U)] == [26, 26, 26, 25]
    team, unit = loops.owner_map(n, T, U, loops.STATIC_CHUNK, 3, loops.TEAMS)
    assert team[:9].tolist() == [0, 0, 0, 1, 1, 1, 2, 2, 2] and (unit == 0).all()
    team, unit = loops.owner_map(n, 1, U, loops.STATIC_CHUNK, 2, loops.UNITS)
    assert unit[:10].tolist() == [0, 0, 1, 1, 2, 2, 3, 3, 0, 0]
    with pytest.raises(ValueError):
        loops.owner_map(n, 2, U, loops.STATIC, 0, loops.UNITS)


def _brute_tiled(dims, tile, T, U, policy, chunk):
    """Enumerate tiles by nested loops over tile coordinates, then points
    inside each tile by nested loops; deal tiles to teams and 4-point groups
    to units."""
    d = len(dims)
    ranges = []
    for (lb, ub, _), tl in zip(dims, tile):
        ranges.append(range(lb // tl, -(-ub // tl)))
    tiles = list(itertools.product(*ranges))
    blocks = _deal_blocks(len(tiles), T)
    owner = {}
    for m, tc in enumerate(tiles):
        if policy == loops.STATIC:
            t = next(i for i, (lo, hi) in enumerate(blocks) if lo <= m < hi)
        else:
            t = (m // chunk) % T
        box = [range(c * tl, (c + 1) * tl) for c, tl in zip(tc, tile)]
        for p, pt in enumerate(itertools.product(*box)):
            if all(lb <= v < ub for v, (lb, ub, _) in zip(pt, dims)):
                owner[pt] = (t, (p // 4) % U)
    pts = loops.serial_iterations(dims)
    return [owner[p][0] for p in pts], [owner[p][1] for p in pts]


@pytest.mark.parametrize("dims,tile,T,U,policy,chunk", [
    ([(1, 9, 1), (1, 13, 1)], (4, 8), 3, 5, loops.STATIC, 0),
    ([(0, 7, 1), (3, 21, 1)], (2, 4), 4, 3, loops.STATIC_CHUNK, 2),
    ([(2, 5, 1)], (4,), 2, 2, loops.STATIC, 0),
    ([(0, 3, 1), (1, 4, 1), (0, 9, 1)], (2, 2, 4), 5, 7, loops.STATIC_CHUNK, 1),
])
def test_tiled_owner_brute_force(dims, tile, T, U, policy, chunk):
    team, unit = loops.tiled_owner_map(dims, tile, T, U, policy, chunk)
    bt, bu = _brute_tiled(dims, tile, T, U, policy, chunk)
    assert team.tolist() == bt and unit.tolist() == bu
