"""Host logic of the task graph under AddressSanitizer and UBSan (CPU only).

The depend-rule table and the persistent engine's table builder are plain
C++ (no HIP). Here they are compiled with -fsanitize=address,undefined
together with a checker (tests/host/engine_tables_check.cpp) that rebuilds
every table directly and compares, and run on:

* the batched workload at its full size (2048 tasks, lengths up to 2^22,
  4051 depend edges, default tiles), with each task's buffers at distinct
  addresses as on the device: predecessors must equal the oracle's depend
  rules (paper sec. 3.3) and every task's data is private to it;
* graphs whose tasks share data (an AXPY chain through y, a reader of
  another task's output, taskloop-style blocks of one array), where exactly
  the tasks that touch another task's data must use coherent accesses;
* degenerate graphs: no tasks, empty loops, inout / repeated addresses.
"""
import os
import shutil
import subprocess

import pytest

import synth
from oracle import tasks as otasks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2209_10643_amd", "csrc")
AXPY, SUM, MATVEC, COVER = 1, 2, 7, 9
DEP_IN, DEP_OUT, DEP_INOUT = 1, 2, 3
MEM_COHERENT = 0

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("asan") / "engine_tables_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "task_graph.cpp"), os.path.join(ROOT, "tests", "host", "engine_tables_check.cpp"),
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


class Addr:
    """Distinct, 256-byte aligned fake device addresses."""

    def __init__(self):
        self.next = 1 << 40

    def take(self, nbytes):
        a = self.next
        self.next += (nbytes + 255) // 256 * 256 + 256
        return a


def run(checker, tmp_path, tasks):
    """tasks: dicts with kind, n, lb, step, tile, red, x, y, A, cols, lda, deps."""
    src, dst = tmp_path / "tasks.txt", tmp_path / "preds.txt"
    with open(src, "w") as f:
        f.write(f"{len(tasks)}\n")
        for t in tasks:
            deps = " ".join(f"{typ} {addr}" for addr, typ in t["deps"])
            f.write(f"{t['kind']} {t['n']} {t.get('lb', 0)} {t.get('step', 1)} {t['tile']} {t.get('red', 0)} "
                    f"{t.get('x', 0)} {t.get('y', 0)} {t.get('A', 0)} {t.get('cols', 0)} {t.get('lda', 0)} "
                    f"{len(t['deps'])} {deps}\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([checker, str(src), str(dst)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    preds = [[int(v) for v in line.split()] for line in open(dst).read().splitlines()]
    info = {}
    for line in r.stdout.splitlines():
        parts = line.split()
        for k, v in zip(parts[::2], parts[1::2]):
            info[k] = int(v)
    return preds, info


def oracle_deps(tasks):
    name = {DEP_IN: otasks.IN, DEP_OUT: otasks.OUT, DEP_INOUT: otasks.INOUT}
    return [[(addr, name[typ]) for addr, typ in t["deps"]] for t in tasks]


def test_full_size_batched_workload(checker, tmp_path):
    seed, n = 12345, 2048
    kinds, lens, preds = synth.batched_spec(seed, n)
    mem, tok = Addr(), (1 << 36)
    tasks = []
    for j, (k, L) in enumerate(zip(kinds, lens)):
        deps = [(tok + 8 * j, DEP_OUT)] + [(tok + 8 * i, DEP_IN) for i in preds[j]]
        if k == "axpy":
            tasks.append(dict(kind=AXPY, n=L, tile=16384, x=mem.take(4 * L), y=mem.take(4 * L), deps=deps))
        elif k == "sum":
            tasks.append(dict(kind=SUM, n=L, tile=16384, red=1, x=mem.take(4 * L), deps=deps))
        else:
            rows = synth.batched_rows(L)
            tasks.append(dict(kind=MATVEC, n=rows, tile=64, A=mem.take(4 * rows * 256), x=mem.take(1024),
                              y=mem.take(4 * rows), cols=256, lda=256, deps=deps))
    got, info = run(checker, tmp_path, tasks)
    assert got == preds == otasks.depend_edges(oracle_deps(tasks))
    assert info["tasks"] == n and info["edges"] == 4051
    assert info["private_tasks"] == n  # every buffer belongs to one task
    want_tiles = sum(max(1, -(-t["n"] // t["tile"])) for t in tasks)
    assert info["tiles"] == want_tiles


def test_shared_data_takes_coherent_accesses(checker, tmp_path):
    mem = Addr()
    n = 5000
    x0, y0 = mem.take(4 * n), mem.take(4 * n)
    xa, ya = mem.take(4 * n), mem.take(4 * n)
    big = mem.take(4 * 4 * n)
    tasks = [
        # 0, 1: an AXPY chain through y0 (both write it)
        dict(kind=AXPY, n=n, tile=1000, x=x0, y=y0, deps=[(y0, DEP_INOUT)]),
        dict(kind=AXPY, n=n, tile=1000, x=x0, y=y0, deps=[(y0, DEP_INOUT)]),
        # 2: reads y0 (written by 0 and 1)
        dict(kind=SUM, n=n, tile=1000, red=1, x=y0, deps=[(y0, DEP_IN)]),
        # 3: AXPY on xa, ya
        dict(kind=AXPY, n=n, tile=1000, x=xa, y=ya, deps=[]),
        # 4-7: taskloop-style disjoint blocks of one array: private
        *[dict(kind=COVER, n=n, tile=1000, y=big + 4 * b * n, deps=[]) for b in range(4)],
        # 8: reads xa, which task 9 writes
        dict(kind=SUM, n=n, tile=1000, red=1, x=xa, deps=[]),
        # 9: a matvec whose output overlaps task 3's x: task 9 writes what 3 reads
        dict(kind=MATVEC, n=4, tile=64, A=mem.take(4 * 4 * 256), x=mem.take(1024), y=xa + 8, cols=256, lda=256,
             deps=[]),
    ]
    got, info = run(checker, tmp_path, tasks)  # the checker compares each mode with a pairwise scan
    assert got == otasks.depend_edges(oracle_deps(tasks))
    # shared: 0, 1, 2 (y0), 3 (reads xa, written by 9), 8 (reads xa), 9; private: the four COVER blocks
    assert info["private_tasks"] == 4


def test_degenerate_graphs(checker, tmp_path):
    assert run(checker, tmp_path, [])[0] == []
    mem = Addr()
    a, b = mem.take(64), mem.take(64)
    tasks = [
        dict(kind=AXPY, n=0, tile=16384, x=a, y=b, deps=[(a, DEP_OUT), (a, DEP_OUT)]),
        dict(kind=SUM, n=1, tile=1, red=2, x=a, deps=[(a, DEP_IN), (b, DEP_INOUT), (a, DEP_IN)]),
        dict(kind=AXPY, n=7, tile=3, x=a, y=b, deps=[(b, DEP_IN)]),
        dict(kind=MATVEC, n=3, tile=1, A=mem.take(3 * 1024), x=mem.take(1024), y=mem.take(12), cols=256,
             lda=256, deps=[(a, DEP_INOUT), (b, DEP_OUT)]),
        dict(kind=SUM, n=(1 << 31) + 5, tile=1 << 30, red=1, x=mem.take(4 * ((1 << 31) + 5)), deps=[(b, DEP_IN)]),
    ]
    got, info = run(checker, tmp_path, tasks)
    assert got == otasks.depend_edges(oracle_deps(tasks))
    assert info["tiles"] == 1 + 1 + 2 + 3 + 129  # tile 3 -> 4; 2^30 -> clamped to 2^24
