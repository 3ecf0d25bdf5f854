"""Reduction operators (serial definitions).

Paper: sec. 5, the synchronization grammar figure lists ``reduction`` among
the collective sync operations, with an operation field ("e.g. add for
add-reduction") and the data it acts on; sec. 3.1 notes that a compiler can
fuse a reduction with the barrier of an SPMD region. The operators offered
here are sum, max and min over all units, with an initial value folded in.
Integer sums are exact in int64; float sums are the correctly rounded exact
sum (``math.fsum``); max and min are exact in any order.
"""
from __future__ import annotations

import math

import numpy as np

SUM, MAX, MIN = "sum", "max", "min"


def reduce(op: str, values, init: float | int | None = None):
    v = np.asarray(values)
    if np.issubdtype(v.dtype, np.integer):
        vals = [int(t) for t in v.ravel().tolist()]
        if op == SUM:
            return (0 if init is None else int(init)) + sum(vals)
        pool = vals + ([] if init is None else [int(init)])
        if not pool:
            return None
        return max(pool) if op == MAX else min(pool)
    vals = np.asarray(v, np.float64).ravel().tolist()
    if op == SUM:
        return math.fsum(vals + ([] if init is None else [float(init)]))
    pool = vals + ([] if init is None else [float(init)])
    if not pool:
        return None
    return max(pool) if op == MAX else min(pool)
