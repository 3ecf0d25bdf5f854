"""Thin conveniences over the C ABI (marshalling only).

Builds the C descriptors from Python values and calls the ``upir_*``
functions; torch tensors supply device memory and the stream.
"""
from __future__ import annotations

import ctypes as C

from . import upir as U


def dev_ptr(t) -> int:
    """Device address of a torch tensor (or an int address)."""
    return t if isinstance(t, int) else t.data_ptr()


def make_loop(dims):
    """dims: list of (lb, ub, step) -> upir_loop."""
    L = U.upir_loop()
    L.collapse = len(dims)
    for d, (lb, ub, st) in enumerate(dims):
        L.dim[d].lb, L.dim[d].ub, L.dim[d].step = int(lb), int(ub), int(st)
    return L


def make_sched(policy=U.UPIR_SCHED_AUTO, chunk=0, distribute=U.UPIR_DIST_TEAMS_UNITS, tile=(0, 0, 0)):
    S = U.upir_sched()
    S.policy, S.chunk, S.distribute = policy, int(chunk), distribute
    t = list(tile) + [0] * (3 - len(tile))
    S.tile[0], S.tile[1], S.tile[2] = (int(v) for v in t[:3])
    return S


def make_spmd(teams=0, units=0, target=U.UPIR_TARGET_GPU):
    return U.upir_spmd(int(teams), int(units), target)


def make_red(op, result, on_host=False, init=0.0, async_=False):
    R = U.upir_reduction()
    R.op, R.result_on_host, R.init, R.async_ = op, int(on_host), float(init), int(async_)
    R.result = result
    return R


class Context:
    """Owns one upir_ctx. ``stream`` is a torch stream (or None)."""

    def __init__(self, device=0, stream=None):
        self.h = C.c_void_p()
        s = None
        if stream is not None:
            s = C.c_void_p(stream.cuda_stream)
        U.upir_init(device, s, C.byref(self.h))
        self._keep = []  # ctypes objects the library may still reference

    def close(self):
        if self.h:
            U.upir_finalize(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------- loops
    def loop(self, kind, args, dims, sched=None, red=None, device_ptrs=True):
        body = U.upir_body(kind, 1 if device_ptrs else 0, C.cast(C.pointer(args), C.c_void_p), C.sizeof(args))
        h = C.c_void_p()
        L = make_loop(dims)
        U.upir_loop_parallel(self.h, C.byref(L), C.byref(sched) if sched is not None else None, C.byref(body),
                             C.byref(red) if red is not None else None, C.byref(h))
        return h

    def launch(self, loops, spmd=None):
        if not isinstance(loops, (list, tuple)):
            loops = [loops]
        arr = (C.c_void_p * len(loops))(*[h.value if isinstance(h, C.c_void_p) else h for h in loops])
        U.upir_spmd_launch(self.h, C.byref(spmd) if spmd is not None else None, arr, len(loops))

    def resolve(self, loop, spmd=None):
        sp, sc, v = U.upir_spmd(), U.upir_sched(), C.c_int32()
        U.upir_loop_resolve(self.h, C.byref(spmd) if spmd is not None else None, loop, C.byref(sp), C.byref(sc),
                            C.byref(v))
        return sp, sc, v.value

    def free(self, loop):
        U.upir_loop_free(self.h, loop)

    def sync(self):
        U.upir_sync(self.h)

    # ------------------------------------------------------------ graphs
    def graph_begin(self):
        U.upir_graph_begin(self.h)

    def graph_end(self):
        g = C.c_void_p()
        U.upir_graph_end(self.h, C.byref(g))
        return g

    def graph_launch(self, g):
        U.upir_graph_launch(self.h, g)

    def graph_destroy(self, g):
        U.upir_graph_destroy(self.h, g)

    # ------------------------------------------------------------- tasks
    def task(self, loop, deps=(), spmd=None):
        arr = (U.upir_depend * max(1, len(deps)))()
        for i, (addr, typ) in enumerate(deps):
            arr[i].addr, arr[i].type = addr, typ
        tid = C.c_int64()
        U.upir_task(self.h, C.byref(spmd) if spmd is not None else None, loop, arr, len(deps), C.byref(tid))
        return tid.value

    def taskloop(self, loop, grainsize=0, num_tasks=0, deps=(), spmd=None):
        """Returns (first task id, number of tasks)."""
        arr = (U.upir_depend * max(1, len(deps)))()
        for i, (addr, typ) in enumerate(deps):
            arr[i].addr, arr[i].type = addr, typ
        first, cnt = C.c_int64(), C.c_int64()
        U.upir_taskloop(self.h, C.byref(spmd) if spmd is not None else None, loop, grainsize, num_tasks, arr,
                        len(deps), C.byref(first), C.byref(cnt))
        return first.value, cnt.value

    def task_update(self, host, nbytes, direction, deps=()):
        """data_update as a task (runs on the copy queue at taskwait PLAIN)."""
        arr = (U.upir_depend * max(1, len(deps)))()
        for i, (addr, typ) in enumerate(deps):
            arr[i].addr, arr[i].type = addr, typ
        tid = C.c_int64()
        U.upir_task_update(self.h, host, nbytes, direction, arr, len(deps), C.byref(tid))
        return tid.value

    def task_preds(self, tid):
        cnt = C.c_int32()
        U.upir_task_preds(self.h, tid, None, 0, C.byref(cnt))
        buf = (C.c_int64 * max(1, cnt.value))()
        U.upir_task_preds(self.h, tid, buf, cnt.value, C.byref(cnt))
        return [buf[i] for i in range(cnt.value)]

    def set_trace(self, tokens=None, start=None, done=None):
        t = U.upir_task_trace(tokens, start, done)
        U.upir_set_task_trace(self.h, C.byref(t))

    def taskwait(self, mode=U.UPIR_TASKWAIT_PLAIN):
        U.upir_taskwait(self.h, mode)

    def taskwait_graph(self, mode=U.UPIR_TASKWAIT_BATCHED):
        g = C.c_void_p()
        U.upir_taskwait_graph(self.h, mode, C.byref(g))
        return g
