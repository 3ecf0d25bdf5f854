"""C ABI checks that need no GPU: the library loads, exports every symbol
the header declares, and its host logic (descriptor validation, data table
bookkeeping, depend -> task graph) behaves as documented.

A host-only context (UPIR_DEVICE_NONE) with a host allocator hook lets the
validation and bookkeeping run without a device; nothing is computed here.
"""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import tasks as otasks
from paper_2209_10643_amd import helpers as H
from paper_2209_10643_amd import upir as U

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "upir.h")

_libc = C.CDLL(None)
_libc.malloc.restype = C.c_void_p
_libc.malloc.argtypes = [C.c_size_t]
_libc.free.argtypes = [C.c_void_p]
_allocs = {"live": 0, "fail": False}


@U.ALLOC_FN
def _host_alloc(n, user):
    if _allocs["fail"]:
        return None
    _allocs["live"] += 1
    return _libc.malloc(n)


@U.FREE_FN
def _host_free(p, user):
    _allocs["live"] -= 1
    _libc.free(p)


def header_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(upir_[a-z0-9_]+)\s*\(", txt)) - {"upir_alloc_fn", "upir_free_fn"})


def test_header_symbols_are_exported():
    names = header_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", U.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(names) == set(U.exported_symbols())
    U.lib()
    assert b"gfx950" in U.upir_version()


@pytest.fixture
def hctx():
    h = C.c_void_p()
    U.upir_init(U.UPIR_DEVICE_NONE, None, C.byref(h))
    U.upir_set_allocator(h, _host_alloc, _host_free, None)
    yield h
    U.upir_finalize(h)
    assert _allocs["live"] == 0


def _status(fn, *args):
    return U.raw(fn)(*args)


def _loop_status(h, dims, kind=U.UPIR_BODY_AXPY, args=None, sched=None, red=None):
    if args is None:
        args = U.upir_axpy_args(2.5, 0, 0x1000, 0x2000)
    body = U.upir_body(kind, 1, C.cast(C.pointer(args), C.c_void_p), C.sizeof(args))
    L = H.make_loop(dims)
    out = C.c_void_p()
    st = _status("upir_loop_parallel", h, C.byref(L), C.byref(sched) if sched else None, C.byref(body),
                 C.byref(red) if red else None, C.byref(out))
    if st == 0:
        U.upir_loop_free(h, out)
    return st


def test_loop_validation(hctx):
    h = hctx
    assert _loop_status(h, [(0, 100, 1)]) == U.UPIR_OK
    assert _loop_status(h, [(0, 100, 0)]) == U.UPIR_EINVAL                  # step 0
    assert _loop_status(h, [(0, 4, 1)] * 2) == U.UPIR_EINVAL                 # AXPY is 1-D
    S = H.make_sched(U.UPIR_SCHED_STATIC_CHUNK, 0)
    assert _loop_status(h, [(0, 100, 1)], sched=S) == U.UPIR_EINVAL          # chunk 0
    S = H.make_sched(U.UPIR_SCHED_STATIC, tile=(6,))
    assert _loop_status(h, [(0, 100, 1)], sched=S) == U.UPIR_EINVAL          # inner tile % 4
    S = H.make_sched(U.UPIR_SCHED_STATIC, tile=(8,))
    assert _loop_status(h, [(0, 100, 2)], sched=S) == U.UPIR_EUNSUPPORTED    # tiled needs unit step
    S = H.make_sched(U.UPIR_SCHED_DYNAMIC, 4, tile=(8,))
    assert _loop_status(h, [(0, 100, 1)], sched=S) == U.UPIR_EUNSUPPORTED
    S = H.make_sched(9)
    assert _loop_status(h, [(0, 100, 1)], sched=S) == U.UPIR_EINVAL
    sa = U.upir_sum_args(0x1000, U.UPIR_DT_F32, 0)
    assert _loop_status(h, [(0, 10, 1)], U.UPIR_BODY_SUM, sa) == U.UPIR_EINVAL  # SUM needs a reduction
    R = H.make_red(U.UPIR_RED_SUM, 0x3000)
    assert _loop_status(h, [(0, 10, 1)], U.UPIR_BODY_SUM, sa, red=R) == U.UPIR_OK
    ow = U.upir_owner_args(0x1000)
    assert _loop_status(h, [(0, 10, 1)], U.UPIR_BODY_OWNER, ow, red=R) == U.UPIR_EINVAL
    assert _loop_status(h, [(0, 3, 1), (0, 4, 1), (2, 9, 3)], U.UPIR_BODY_OWNER, ow) == U.UPIR_OK
    assert _loop_status(h, [(0, 3, 1)] * 4 if False else [(0, 3, 1)], 42) == U.UPIR_EINVAL  # unknown body
    mm = U.upir_matmul_args(0x1000, 0x2000, 0x3000, 8, 4, 16, 16, None, 0)   # lda < K
    assert _loop_status(h, [(0, 16, 1), (0, 16, 1)], U.UPIR_BODY_MATMUL_F32, mm) == U.UPIR_EINVAL
    mm = U.upir_matmul_args(0x1000, 0x2000, 0x3000, 8, 8, 16, 16, None, 0)
    assert _loop_status(h, [(1, 16, 1), (0, 16, 1)], U.UPIR_BODY_MATMUL_F32, mm) == U.UPIR_EUNSUPPORTED
    assert _loop_status(h, [(0, 16, 1), (0, 16, 1)], U.UPIR_BODY_MATMUL_F32, mm) == U.UPIR_OK
    f7 = U.upir_filter7_args(0x1000, 0x2000, 0x3000, 64)
    assert _loop_status(h, [(3, 61, 1), (3, 61, 1)], U.UPIR_BODY_FILTER7, f7) == U.UPIR_OK
    assert _loop_status(h, [(3, 61, 1)], U.UPIR_BODY_FILTER7, f7) == U.UPIR_EINVAL            # 2-D only
    assert _loop_status(h, [(3, 61, 1)] * 2, U.UPIR_BODY_FILTER7, f7, red=R) == U.UPIR_EINVAL  # no reduction
    f7 = U.upir_filter7_args(0x1000, 0x2000, 0x3000, 0)
    assert _loop_status(h, [(3, 61, 1)] * 2, U.UPIR_BODY_FILTER7, f7) == U.UPIR_EINVAL        # pitch


def test_launch_needs_device(hctx):
    h = hctx
    args = U.upir_axpy_args(2.5, 0, 0x1000, 0x2000)
    body = U.upir_body(U.UPIR_BODY_AXPY, 1, C.cast(C.pointer(args), C.c_void_p), C.sizeof(args))
    L = H.make_loop([(0, 8, 1)])
    lp = C.c_void_p()
    U.upir_loop_parallel(h, C.byref(L), None, C.byref(body), None, C.byref(lp))
    arr = (C.c_void_p * 1)(lp.value)
    assert _status("upir_spmd_launch", h, None, arr, 1) == U.UPIR_ESTATE
    assert _status("upir_graph_begin", h) == U.UPIR_ESTATE
    assert _status("upir_sync", h) == U.UPIR_ESTATE
    assert b"host-only" in U.upir_last_error(h)
    U.upir_loop_free(h, lp)


def test_data_table_bookkeeping(hctx):
    h = hctx
    buf = (C.c_float * 64)()
    base = C.addressof(buf)
    d0 = C.c_void_p()
    U.upir_data_map(h, base, 256, U.UPIR_MAP_ALLOC, U.UPIR_ACCESS_RW, C.byref(d0))
    # a sub-range is present: reference count grows, same device memory
    d1 = C.c_void_p()
    U.upir_data_map(h, base + 16, 32, U.UPIR_MAP_ALLOC, U.UPIR_ACCESS_RW, C.byref(d1))
    assert d1.value == d0.value + 16
    look = C.c_void_p()
    U.upir_data_lookup(h, base + 100, C.byref(look))
    assert look.value == d0.value + 100
    # partial overlap is refused
    assert _status("upir_data_map", h, base + 200, 100, U.UPIR_MAP_ALLOC, U.UPIR_ACCESS_RW, None) == U.UPIR_EOVERLAP
    assert _status("upir_data_map", h, base - 8, 16, U.UPIR_MAP_ALLOC, U.UPIR_ACCESS_RW, None) == U.UPIR_EOVERLAP
    # copies need a device
    other = (C.c_float * 4)()
    assert _status("upir_data_map", h, C.addressof(other), 16, U.UPIR_MAP_TO, U.UPIR_ACCESS_RO, None) == U.UPIR_ESTATE
    # bad arguments
    assert _status("upir_data_map", h, None, 16, U.UPIR_MAP_ALLOC, U.UPIR_ACCESS_RW, None) == U.UPIR_EINVAL
    assert _status("upir_data_map", h, base, 16, 9, U.UPIR_ACCESS_RW, None) == U.UPIR_EINVAL
    # unmap: only the start of a mapping; two references -> two unmaps
    assert _status("upir_data_unmap", h, base + 4, U.UPIR_MAP_ALLOC) == U.UPIR_ENOTMAPPED
    live = _allocs["live"]
    U.upir_data_unmap(h, base, U.UPIR_MAP_ALLOC)
    assert _allocs["live"] == live                       # still referenced
    U.upir_data_unmap(h, base, U.UPIR_MAP_ALLOC)
    assert _allocs["live"] == live - 1                   # freed through the hook
    assert _status("upir_data_unmap", h, base, U.UPIR_MAP_ALLOC) == U.UPIR_ENOTMAPPED
    assert _status("upir_data_lookup", h, base, C.byref(look)) == U.UPIR_ENOTMAPPED


def test_allocation_failure_leaks_nothing(hctx):
    h = hctx
    buf = (C.c_float * 8)()
    live = _allocs["live"]
    _allocs["fail"] = True
    try:
        assert _status("upir_data_map", h, C.addressof(buf), 32, U.UPIR_MAP_ALLOC, U.UPIR_ACCESS_RW, None) \
            == U.UPIR_ENOMEM
        assert _loop_status(h, [(0, 10, 1)]) == U.UPIR_ENOMEM
    finally:
        _allocs["fail"] = False
    assert _allocs["live"] == live
    # the allocator cannot change while something is allocated
    U.upir_data_map(h, C.addressof(buf), 32, U.UPIR_MAP_ALLOC, U.UPIR_ACCESS_RW, None)
    assert _status("upir_set_allocator", h, _host_alloc, _host_free, None) == U.UPIR_ESTATE
    U.upir_data_unmap(h, C.addressof(buf), U.UPIR_MAP_ALLOC)


def _task_loop(h):
    args = U.upir_cover_args(0x1000)
    body = U.upir_body(U.UPIR_BODY_COVER, 1, C.cast(C.pointer(args), C.c_void_p), C.sizeof(args))
    L = H.make_loop([(0, 16, 1)])
    lp = C.c_void_p()
    U.upir_loop_parallel(h, C.byref(L), None, C.byref(body), None, C.byref(lp))
    return lp


def _add_task(h, lp, deps):
    arr = (U.upir_depend * max(1, len(deps)))()
    for i, (addr, typ) in enumerate(deps):
        arr[i].addr, arr[i].type = addr, typ
    tid = C.c_int64()
    U.upir_task(h, None, lp, arr, len(deps), C.byref(tid))
    return tid.value


def _preds(h, tid):
    cnt = C.c_int32()
    buf = (C.c_int64 * 4096)()
    U.upir_task_preds(h, tid, buf, 4096, C.byref(cnt))
    return [buf[i] for i in range(cnt.value)]


TYPES = {U.UPIR_DEP_IN: otasks.IN, U.UPIR_DEP_OUT: otasks.OUT, U.UPIR_DEP_INOUT: otasks.INOUT}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_depend_graph_matches_oracle(hctx, seed):
    h = hctx
    lp = _task_loop(h)
    rng = np.random.default_rng(seed)
    n = 60
    deps = []
    for j in range(n):
        k = int(rng.integers(0, 4))
        dl = [(int(rng.integers(1, 9)) * 64, int(rng.integers(1, 4))) for _ in range(k)]
        deps.append(dl)
        assert _add_task(h, lp, dl) == j
    want = otasks.depend_edges([[(a, TYPES[t]) for a, t in dl] for dl in deps])
    got = [_preds(h, j) for j in range(n)]
    assert got == want
    # the batched workload's encoding: out on tok[j], in on tok[i]
    assert _status("upir_taskwait", h, U.UPIR_TASKWAIT_PLAIN) == U.UPIR_ESTATE


def _cover_loop(h, n, lb=0):
    args = U.upir_cover_args(0x1000)
    body = U.upir_body(U.UPIR_BODY_COVER, 1, C.cast(C.pointer(args), C.c_void_p), C.sizeof(args))
    L = H.make_loop([(lb, lb + n, 1)])
    lp = C.c_void_p()
    U.upir_loop_parallel(h, C.byref(L), None, C.byref(body), None, C.byref(lp))
    return lp


def _add_taskloop(h, lp, deps, g=0, k=0):
    arr = (U.upir_depend * max(1, len(deps)))()
    for i, (addr, typ) in enumerate(deps):
        arr[i].addr, arr[i].type = addr, typ
    first, cnt = C.c_int64(), C.c_int64()
    U.upir_taskloop(h, None, lp, g, k, arr, len(deps), C.byref(first), C.byref(cnt))
    return first.value, cnt.value


@pytest.mark.parametrize("seed", [0, 1])
def test_taskloop_graph_matches_oracle(hctx, seed):
    """Random mixes of tasks and taskloops: task counts from grainsize /
    num_tasks and every predecessor list, against the oracle's rules."""
    h = hctx
    rng = np.random.default_rng(seed)
    loops = {n: _cover_loop(h, n) for n in (1, 7, 100, 1000, 65537)}
    deps, groups, ntasks = [], [], 0
    for step in range(40):
        dl = [(int(rng.integers(1, 7)) * 64, int(rng.integers(1, 4))) for _ in range(int(rng.integers(0, 3)))]
        odl = [(a, TYPES[t]) for a, t in dl]
        if rng.random() < 0.5:
            n = int(rng.choice(list(loops)))
            g, k = [(7, 0), (0, 5), (30, 4), (0, 0), (1000, 0)][int(rng.integers(0, 5))]
            first, cnt = _add_taskloop(h, loops[n], dl, g, k)
            assert first == ntasks
            assert cnt == otasks.taskloop_count(n, g, k, default=max(1, -(-n // 65536)))
            deps += [odl] * cnt
            groups += [step] * cnt
            ntasks += cnt
        else:
            assert _add_task(h, loops[7], dl) == ntasks
            deps.append(odl)
            groups.append(None)
            ntasks += 1
    want = otasks.depend_edges(deps, groups)
    assert [_preds(h, j) for j in range(ntasks)] == want


def test_taskloop_validation(hctx):
    h = hctx
    lp = _cover_loop(h, 100)
    first, cnt = C.c_int64(), C.c_int64()
    assert _status("upir_taskloop", h, None, lp, -1, 0, None, 0, C.byref(first), C.byref(cnt)) == U.UPIR_EINVAL
    sa = U.upir_sum_args(0x1000, U.UPIR_DT_F32, 0)
    body = U.upir_body(U.UPIR_BODY_SUM, 1, C.cast(C.pointer(sa), C.c_void_p), C.sizeof(sa))
    L = H.make_loop([(0, 100, 1)])
    R = H.make_red(U.UPIR_RED_SUM, 0x3000)
    sl = C.c_void_p()
    U.upir_loop_parallel(h, C.byref(L), None, C.byref(body), C.byref(R), C.byref(sl))
    assert _status("upir_taskloop", h, None, sl, 10, 0, None, 0, C.byref(first), C.byref(cnt)) == U.UPIR_EUNSUPPORTED
    empty = _cover_loop(h, 0)
    assert _add_taskloop(h, empty, [], 4, 0) == (0, 0)   # no iterations, no tasks


def test_task_validation(hctx):
    h = hctx
    lp = _task_loop(h)
    bad = (U.upir_depend * 1)()
    bad[0].addr, bad[0].type = 64, 7
    tid = C.c_int64()
    assert _status("upir_task", h, None, lp, bad, 1, C.byref(tid)) == U.UPIR_EDEPEND
    assert _status("upir_task", h, None, lp, None, -1, C.byref(tid)) == U.UPIR_EDEPEND
    sp = H.make_spmd(target=U.UPIR_TARGET_CLUSTER)
    assert _status("upir_task", h, C.byref(sp), lp, None, 0, C.byref(tid)) == U.UPIR_EUNSUPPORTED
    # a jacobi loop is not offered as a task
    ja = U.upir_jacobi5_args(0x1000, 0x2000, 16)
    body = U.upir_body(U.UPIR_BODY_JACOBI5, 1, C.cast(C.pointer(ja), C.c_void_p), C.sizeof(ja))
    L = H.make_loop([(1, 15, 1), (1, 15, 1)])
    jl = C.c_void_p()
    U.upir_loop_parallel(h, C.byref(L), None, C.byref(body), None, C.byref(jl))
    assert _status("upir_task", h, None, jl, None, 0, C.byref(tid)) == U.UPIR_EUNSUPPORTED
    _add_task(h, lp, [])
    assert _status("upir_loop_free", h, lp) == U.UPIR_ESTATE  # in use by a pending task


def test_status_strings():
    for s in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert U.lib().upir_strerror(s)
    assert U.upir_matmul_workspace_bytes(U.UPIR_BODY_MATMUL_SPLIT3, 4096, 4096, 4096) == 2 * 4096 * 4096 * 4
    # k is padded to the 32-wide panels of the four-wavefront tile's layout
    assert U.upir_matmul_workspace_bytes(U.UPIR_BODY_MATMUL_BF16, 17, 33, 65) == (17 + 33) * 96 * 2
    assert U.upir_matmul_workspace_bytes(U.UPIR_BODY_MATMUL_SPLIT3, 17, 33, 64) == (17 + 33) * 64 * 4


def test_update_task_graph_and_validation(hctx):
    """data_update tasks take part in the depend graph like loop tasks."""
    h = hctx
    lp = _cover_loop(h, 16)
    X, Y = 0x100, 0x200
    tid = C.c_int64()
    arr = (U.upir_depend * 1)()
    arr[0].addr, arr[0].type = X, U.UPIR_DEP_OUT
    assert _status("upir_task_update", h, 0x5000, 64, U.UPIR_TO_DEVICE, arr, 1, C.byref(tid)) == U.UPIR_OK
    assert tid.value == 0
    assert _add_task(h, lp, [(X, U.UPIR_DEP_IN), (Y, U.UPIR_DEP_OUT)]) == 1
    arr[0].addr, arr[0].type = Y, U.UPIR_DEP_IN
    assert _status("upir_task_update", h, 0x5000, 64, U.UPIR_FROM_DEVICE, arr, 1, C.byref(tid)) == U.UPIR_OK
    want = otasks.depend_edges([[(X, otasks.OUT)], [(X, otasks.IN), (Y, otasks.OUT)], [(Y, otasks.IN)]])
    assert [_preds(h, j) for j in range(3)] == want == [[], [0], [1]]
    assert _status("upir_task_update", h, 0x5000, 64, 9, None, 0, C.byref(tid)) == U.UPIR_EINVAL
    assert _status("upir_task_update", h, None, 64, U.UPIR_TO_DEVICE, None, 0, C.byref(tid)) == U.UPIR_EINVAL


# Every structure of the C ABI: the C compiler's size and field offsets for
# the header's declaration must equal the ctypes mirror's.
ABI_STRUCTS = ["upir_spmd", "upir_dim", "upir_loop", "upir_sched", "upir_reduction", "upir_axpy_args",
               "upir_sum_args", "upir_jacobi5_args", "upir_matmul_args", "upir_matvec_args", "upir_owner_args",
               "upir_cover_args", "upir_filter7_args", "upir_body", "upir_depend", "upir_task_trace",
               "upir_engine_sched"]
C_FIELD_NAMES = {"async_": "async"}  # a Python keyword renamed in the binding


def test_struct_layouts_match_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "upir.h"', "int main(void) {"]
    for s in ABI_STRUCTS:
        cls = getattr(U, s)
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for name, _ in cls._fields_:
            cname = C_FIELD_NAMES.get(name, name)
            lines.append(f'  printf("{s} {name} %zu\\n", offsetof({s}, {cname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        s, field, v = ln.split()
        got[(s, field)] = int(v)
    for s in ABI_STRUCTS:
        cls = getattr(U, s)
        assert got[(s, "size")] == C.sizeof(cls), s
        for name, _ in cls._fields_:
            assert got[(s, name)] == getattr(cls, name).offset, (s, name)
