"""The batched-task workload at its full size against the oracle.

2048 tasks (AXPY, SUM, MATVEC of 256 columns; lengths floor(2^u), u uniform
in [8, 22]; 4051 random depend edges, two successors per task on average),
run by the persistent engine from a captured graph with the default tiles,
as the benchmark launches it. Every task is compared with the oracle's
serial elision of that task, its inputs regenerated on the host from the
seeded generators (a pool of worker processes, one task at a time each):
AXPY outputs bit-exact, SUM within 1e-5 * sum|x|, MATVEC normwise 1e-5; every
token of the chain equals the oracle's, and every edge i -> j has
done[i] < start[j].
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np
import pytest

import synth
from oracle import bodies, tasks as otasks
from paper_2209_10643_amd import helpers as H
from paper_2209_10643_amd import upir as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED, N_TASKS = 12345, 2048


def note(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.timeout(900)
def test_batched_full_size_matches_oracle():
    assert torch.cuda.is_available()
    U.lib()
    s = torch.cuda.Stream()
    prev = torch.cuda.current_stream()
    torch.cuda.set_stream(s)
    ctx = H.Context(0, stream=s)
    try:
        t0 = time.time()
        kinds, lens, preds = synth.batched_spec(SEED, N_TASKS)
        assert sum(len(p) for p in preds) == 4051
        bufs, handles = [], []
        for j, (kind, L) in enumerate(zip(kinds, lens)):
            d = synth.batched_inputs_torch(SEED, j, kind, L, device="cuda")
            if kind == "axpy":
                h = ctx.loop(U.UPIR_BODY_AXPY, U.upir_axpy_args(2.5, 0, d["x"].data_ptr(), d["y"].data_ptr()),
                             [(0, L, 1)])
            elif kind == "sum":
                d["r"] = torch.zeros(1, dtype=torch.float64, device="cuda")
                h = ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(d["x"].data_ptr(), U.UPIR_DT_F32, 0), [(0, L, 1)],
                             None, H.make_red(U.UPIR_RED_SUM, d["r"].data_ptr()))
            else:
                rows = synth.batched_rows(L)
                d["y"] = torch.zeros(rows, device="cuda")
                h = ctx.loop(U.UPIR_BODY_MATVEC, U.upir_matvec_args(d["A"].data_ptr(), d["x"].data_ptr(),
                                                                     d["y"].data_ptr(), 256, 256), [(0, rows, 1)])
            bufs.append(d)
            handles.append(h)
        tok = torch.zeros(N_TASKS, dtype=torch.int64, device="cuda")
        start = torch.zeros(N_TASKS, dtype=torch.int64, device="cuda")
        done = torch.zeros(N_TASKS, dtype=torch.int64, device="cuda")
        base = tok.data_ptr()
        for j, h in enumerate(handles):
            deps = [(base + 8 * j, U.UPIR_DEP_OUT)] + [(base + 8 * i, U.UPIR_DEP_IN) for i in preds[j]]
            ctx.task(h, deps)
        ctx.set_trace(tok.data_ptr(), start.data_ptr(), done.data_ptr())
        g = ctx.taskwait_graph(U.UPIR_TASKWAIT_BATCHED)
        ctx.set_trace()
        note(f"batched full size: workload on the device in {time.time() - t0:.1f}s; running the engine graph")
        ctx.graph_launch(g)
        ctx.sync()
        ctx.graph_destroy(g)
        note("engine done; comparing with the oracle")
        assert [int(v) & (2 ** 64 - 1) for v in tok.cpu().numpy().tolist()] == otasks.tokens(preds)
        st, dn = start.cpu().numpy(), done.cpu().numpy()
        for j, pj in enumerate(preds):
            for i in pj:
                assert dn[i] < st[j], (i, j)
        jobs = [(SEED, j, kinds[j], lens[j]) for j in range(N_TASKS)]
        workers = max(1, min(16, (os.cpu_count() or 2) - 1))
        checked = {"axpy": 0, "sum": 0, "matvec": 0}
        with mp.get_context("spawn").Pool(workers) as pool:
            for j, (kind, want, l1) in enumerate(pool.imap(otasks.batched_task_expected_job, jobs, chunksize=4)):
                d = bufs[j]
                if kind == "axpy":
                    got = d["y"].cpu().numpy()
                    assert np.array_equal(got, want["y"]), f"task {j} (AXPY, n={lens[j]})"
                elif kind == "sum":
                    got = float(d["r"].item())
                    assert abs(got - want["s"]) <= 1e-5 * l1, f"task {j} (SUM, n={lens[j]})"
                else:
                    got = d["y"].cpu().numpy().astype(np.float64)
                    assert bodies.frob_rel(got, want["y"]) <= 1e-5, f"task {j} (MATVEC, n={lens[j]})"
                checked[kind] += 1
                if j % 256 == 255:
                    note(f"  {j + 1} tasks match the oracle")
        assert sum(checked.values()) == N_TASKS
        note(f"batched full size: all {N_TASKS} tasks match ({checked}) in {time.time() - t0:.1f}s")
        for h in handles:
            ctx.free(h)
    finally:
        ctx.close()
        torch.cuda.set_stream(prev)
