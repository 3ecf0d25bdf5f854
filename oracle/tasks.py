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


def depend_edges(deps, groups=None):
    """Predecessor sets from per-task depend lists.

    ``deps[j]`` is a list of (address, type) pairs for task j, in creation
    order. Returns ``preds[j]``, a sorted list of distinct task ids.
    ``groups[j]`` (optional) names the taskloop that generated task j: tasks
    of one taskloop carry the taskloop's depend list and are siblings that do
    not wait for each other (None: a task of its own).
    """
    preds = []
    for j, dl in enumerate(deps):
        p = set()
        for addr, typ in dl:
            for i in range(j):
                if groups is not None and groups[j] is not None and groups[i] == groups[j]:
                    continue
                for addr_i, typ_i in deps[i]:
                    if addr_i != addr:
                        continue
                    if typ == IN and typ_i in (OUT, INOUT):
                        p.add(i)
                    elif typ in (OUT, INOUT):
                        p.add(i)
        preds.append(sorted(p))
    return preds


def taskloop_count(n: int, grainsize: int = 0, num_tasks: int = 0, default: int = 1) -> int:
    """Number of tasks a taskloop makes of ``n`` iterations (sec. 3.2 taskloop
    fields, read as OpenMP's): ``num_tasks(k)`` asks for k tasks (at most one
    per iteration); ``grainsize(g)`` for floor(n / g) tasks, so each has at
    least g iterations (and fewer than 2g); with both, the smaller count;
    with neither, ``default``. No iterations: no tasks."""
    if n <= 0:
        return 0
    cands = []
    if num_tasks > 0:
        cands.append(min(num_tasks, n))
    if grainsize > 0:
        cands.append(max(1, n // grainsize))
    g = min(cands) if cands else min(max(default, 1), n)
    return max(1, g)


def taskloop_blocks(n: int, grainsize: int = 0, num_tasks: int = 0, default: int = 1):
    """The iteration ranges [lo, hi) of a taskloop's tasks, in task order:
    near-equal contiguous blocks, the first n mod G one longer."""
    g = taskloop_count(n, grainsize, num_tasks, default)
    out = []
    q, r = divmod(n, g) if g else (0, 0)
    for t in range(g):
        lo = t * q + min(t, r)
        out.append((lo, lo + q + (1 if t < r else 0)))
    return out


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


def batched_task_expected(seed: int, j: int, kind: str, L: int):
    """Expected result of task j of the seeded batched workload: its inputs
    are regenerated on the host from the seeded generators (nothing comes
    from the GPU) and its loop runs as its serial elision. Returns
    (kind, result dict, sum |x| for SUM tasks else 0.0); a module-level
    function so that a pool of worker processes can run it."""
    import synth  # the seeded input generators (no loop arithmetic)

    args = synth.batched_inputs(seed, j, kind, L)
    res = run_task(kind, args)
    l1 = bodies.sum_abs_f64(args["x"]) if kind == "sum" else 0.0
    return kind, res, l1


def batched_task_expected_job(job):
    """batched_task_expected over one (seed, j, kind, L) tuple (for Pool.imap)."""
    return batched_task_expected(*job)
