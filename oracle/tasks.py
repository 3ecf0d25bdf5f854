"""Tasks with ``depend``: task graph, index-order execution, token chain.

Paper: sec. 3.3 "Asynchronous Task Parallelism", the tasking grammar figure:
a task has depend, data, sync and scheduling-policy fields and may be an
offloaded task (``offload(device: id)``); the depend field is "similar to the
OpenMP depend clause", and an offloaded kernel launch counts as a task. Sec. 5
lists ``taskwait`` among the sync operations.

Reading of "similar to OpenMP depend" (OpenMP 5 task dependences between
sibling tasks, in creation order): a task with ``in`` on address X depends on
every earlier task with ``out`` or ``inout`` on X; a task with ``out`` or
``inout`` on X depends on every earlier task that names X at all. Edges go
from lower to higher creation index, so the graph is acyclic and creation
order is a topological order: the serial elision runs tasks in that order.

The token chain is an observation device of the task engine, not part of the
paper: after task j runs, ``tok[j] = chain(j, tok[p] for p in preds(j))`` with
SplitMix64's finalizer (Steele, Lea, Flood 2014). A task that ran before a
predecessor finished, or read a stale token, yields a different value.
"""
from __future__ import annotations

import numpy as np

from . import bodies

IN, OUT, INOUT = "in", "out", "inout"

_G = 0x9E3779B97F4A7C15
_MASK = (1 << 64) - 1


def _mix64(z: int) -> int:
    """SplitMix64 finalizer (Steele, Lea, Flood 2014), mod 2**64."""
    z &= _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def depend_edges(deps):
    """Predecessor sets from per-task depend lists.

    ``deps[j]`` is a list of (address, type) pairs for task j, in creation
    order. Returns ``preds[j]``, a sorted list of distinct task ids.
    """
    preds = []
    for j, dl in enumerate(deps):
        p = set()
        for addr, typ in dl:
            for i in range(j):
                for addr_i, typ_i in deps[i]:
                    if addr_i != addr:
                        continue
                    if typ == IN and typ_i in (OUT, INOUT):
                        p.add(i)
                    elif typ in (OUT, INOUT):
                        p.add(i)
        preds.append(sorted(p))
    return preds


def tokens(preds):
    """``tok[j] = h`` where ``h = mix64((j+1) G)`` then ``h = mix64(h ^ tok[p])``
    for each predecessor p in ascending order (tasks taken in index order)."""
    tok = []
    for j, pj in enumerate(preds):
        h = _mix64(((j + 1) * _G) & _MASK)
        for p in pj:
            h = _mix64(h ^ tok[p])
        tok.append(h)
    return tok


def run_task(kind: str, args: dict):
    """One task's loop as its serial elision (the bodies of sec. 6)."""
    if kind == "axpy":
        return {"y": bodies.axpy(args["a"], args["x"], args["y"])}
    if kind == "sum":
        return {"s": bodies.sum_f64(args["x"])}
    if kind == "matvec":
        return {"y": bodies.matvec(args["A"], args["x"])}
    raise ValueError(kind)


def run_in_order(tasks):
    """Run a list of (kind, args) tasks in creation (index) order."""
    return [run_task(k, a) for k, a in tasks]
