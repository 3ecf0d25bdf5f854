"""Canonical loops, collapse and worksharing owner maps (serial definitions).

Paper: sec. 3.2 "Data Parallelism", the loop / loop_parallel grammar figure:
a canonical loop has an induction variable, lowerBound, upperBound, step and
collapse(n); loop_parallel worksharing has schedule(static|dynamic|guided|
runtime|auto[, chunk]) and distribute(teams|units|teams,units), and must sit
inside an SPMD region whose units form two levels, teams and units (sec. 3.1).

The paper names the policies but gives no formula; it says worksharing is
"similar to the OpenMP standard". The readings used here:

* upper bound exclusive (the AXPY loop of sec. 6 runs ``i < n``);
* trip count ``ceil((ub - lb) / step)`` for step > 0 and
  ``ceil((lb - ub) / -step)`` for step < 0, never negative;
* collapse linearises the nest row-major (outermost dimension slowest);
* ``static`` without chunk, distribute(teams,units): the ``n`` iterations are
  cut into ``T`` near-equal contiguous blocks, the first ``n % T`` one longer;
  team ``t`` takes block ``t`` and cuts it the same way among its ``U`` units;
* ``static, c``: chunk ``m`` = iterations ``[m c, min((m+1) c, n))`` goes to
  flat unit ``m mod (T U)`` where flat = ``t U + u``;
* distribute(teams): the team level as above, executed by unit 0 of the team;
* distribute(units): one team (``T`` must be 1), units as above;
* tiled schedules (tiling applied before worksharing, which the separation of
  loop and loop_parallel in sec. 3.2 permits): unit steps; tiles anchored at
  induction value 0; tiles are numbered row-major over the tiles that meet the
  iteration box and handed to teams by the policy (static blocks or chunks of
  tiles, cyclic over teams); inside a tile, points are numbered row-major over
  the full tile box, and group ``p // 4`` of four consecutive points goes to
  unit ``(p // 4) mod U``.
"""
from __future__ import annotations

import numpy as np

STATIC, STATIC_CHUNK = "static", "static_chunk"
TEAMS, UNITS, TEAMS_UNITS = "teams", "units", "teams_units"
UNIT_GROUP = 4   # consecutive points per unit slice inside a tile


def trip_count(lb: int, ub: int, step: int) -> int:
    """Iterations of ``for (i = lb; i <op> ub; i += step)``, ub exclusive."""
    if step == 0:
        raise ValueError("step must be non-zero")
    if step > 0:
        return max(0, -(-(ub - lb) // step))
    return max(0, -(-(lb - ub) // (-step)))


def collapse_decode(dims, k: int):
    """Induction values of collapsed iteration ``k`` (row-major order)."""
    counts = [trip_count(*d) for d in dims]
    idx = []
    for c in reversed(counts):
        idx.append(k % c)
        k //= c
    idx.reverse()
    return tuple(lb + i * st for (lb, _, st), i in zip(dims, idx))


def serial_iterations(dims):
    """The serial elision: induction tuples in index order (nested loops)."""
    out = [()]
    for lb, ub, st in dims:
        vals = [lb + i * st for i in range(trip_count(lb, ub, st))]
        out = [t + (v,) for t in out for v in vals]
    return out


def block(n: int, parts: int, p: int):
    """Block ``p`` of ``n`` items cut into ``parts`` near-equal pieces."""
    q, r = divmod(n, parts)
    lo = p * q + min(p, r)
    return lo, lo + q + (1 if p < r else 0)


def owner_map(n: int, T: int, U: int, policy: str = STATIC, chunk: int = 0,
              distribute: str = TEAMS_UNITS):
    """(team[k], unit[k]) for every collapsed iteration ``k`` of an untiled loop.

    Written block by block from the definitions above, so a reader can check
    it by eye; a test checks it against per-iteration brute force.
    """
    team = np.full(n, -1, dtype=np.int64)
    unit = np.full(n, -1, dtype=np.int64)
    if distribute == UNITS and T != 1:
        raise ValueError("distribute(units) runs on one team")
    if policy == STATIC:
        for t in range(T):
            tlo, thi = block(n, T, t)
            if distribute == TEAMS:
                team[tlo:thi], unit[tlo:thi] = t, 0
                continue
            for u in range(U):
                ulo, uhi = block(thi - tlo, U, u)
                team[tlo + ulo:tlo + uhi] = t
                unit[tlo + ulo:tlo + uhi] = u
    elif policy == STATIC_CHUNK:
        if chunk <= 0:
            raise ValueError("chunk must be positive")
        for m in range(-(-n // chunk)):
            lo, hi = m * chunk, min((m + 1) * chunk, n)
            if distribute == TEAMS_UNITS:
                f = m % (T * U)
                team[lo:hi], unit[lo:hi] = f // U, f % U
            elif distribute == TEAMS:
                team[lo:hi], unit[lo:hi] = m % T, 0
            else:
                team[lo:hi], unit[lo:hi] = 0, m % U
    else:
        raise ValueError(policy)
    return team, unit


def tiled_owner_map(dims, tile, T: int, U: int, policy: str = STATIC, chunk: int = 0):
    """(team[k], unit[k]) for a tiled loop nest, k the collapsed index.

    ``dims`` is a list of (lb, ub, 1); ``tile`` the tile extent per dimension.
    """
    d = len(dims)
    for lb, ub, st in dims:
        if st != 1:
            raise ValueError("tiled schedules need unit steps")
    counts = [trip_count(*x) for x in dims]
    n = int(np.prod(counts)) if counts else 0
    t0 = [lb // tl for (lb, _, _), tl in zip(dims, tile)]                 # first tile coord
    nt = [-(-ub // tl) - a for (_, ub, _), tl, a in zip(dims, tile, t0)]  # tiles per dim
    ntiles = int(np.prod(nt))
    # team of each tile
    tile_team = np.empty(ntiles, dtype=np.int64)
    if policy == STATIC:
        for t in range(T):
            lo, hi = block(ntiles, T, t)
            tile_team[lo:hi] = t
    elif policy == STATIC_CHUNK:
        for m in range(ntiles):
            tile_team[m] = (m // chunk) % T
    else:
        raise ValueError(policy)
    team = np.empty(n, dtype=np.int64)
    unit = np.empty(n, dtype=np.int64)
    for k in range(n):
        iv = collapse_decode(dims, k)
        tc = [v // tl for v, tl in zip(iv, tile)]
        m = 0
        for j in range(d):
            m = m * nt[j] + (tc[j] - t0[j])
        p = 0
        for j in range(d):
            p = p * tile[j] + (iv[j] - tc[j] * tile[j])
        team[k] = tile_team[m]
        unit[k] = (p // UNIT_GROUP) % U
    return team, unit
