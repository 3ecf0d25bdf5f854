"""GPU parity of tasks with depend: plain (one launch per task) and batched
(one persistent kernel) executors against the oracle's index-order run.

Bit-exact: AXPY outputs, MATVEC outputs between the two executors, tokens
(the chain over each task's predecessors, which a stale read or a violated
edge would change), coverage counts. Stamps: every edge i -> j has
done[i] < start[j]. SUM results within 1e-5 * sum|x|, MATVEC normwise 1e-5.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import synth
from oracle import bodies, tasks as otasks
from paper_2209_10643_amd import helpers as H
from paper_2209_10643_amd import upir as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def note(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    U.lib()
    s = torch.cuda.Stream()
    prev = torch.cuda.current_stream()
    torch.cuda.set_stream(s)  # torch's work and the library's are ordered on one stream
    c = H.Context(0, stream=s)
    yield c
    c.close()
    torch.cuda.set_stream(prev)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_workload(seed, n, lmin=8, lmax=16, p_edge=None):
    """The seeded batched recipe (kinds uniform over AXPY / SUM / MATVEC,
    lengths floor(2^u) with u uniform in [lmin, lmax], edges i < j with
    probability 4/(n-1)) at a reduced size, with host inputs."""
    kinds, lens, preds = synth.batched_spec(seed, n, lmin, lmax, p_edge)
    specs = [(k, synth.batched_inputs(seed, j, k, L)) for j, (k, L) in enumerate(zip(kinds, lens))]
    return specs, preds


def build_tasks(ctx, specs, preds, tile=0):
    """tile: 0 for the default (AUTO) schedule, n > 0 for AUTO with an n-element
    tile, "static" for a STATIC schedule without a tile (the engine then
    takes its default tiles rather than the graph's engine schedule)."""
    tok = torch.zeros(len(specs), dtype=torch.int64, device="cuda")
    handles, bufs = [], []
    if tile == "static":
        sched = H.make_sched(U.UPIR_SCHED_STATIC)
    else:
        sched = H.make_sched(U.UPIR_SCHED_AUTO, tile=(tile,)) if tile else None
    for j, (kind, a) in enumerate(specs):
        if kind == "axpy":
            tx, ty = dev(a["x"]), dev(a["y"])
            args = U.upir_axpy_args(2.5, 0, tx.data_ptr(), ty.data_ptr())
            lp = ctx.loop(U.UPIR_BODY_AXPY, args, [(0, len(a["x"]), 1)], sched)
            bufs.append((tx, ty))
        elif kind == "sum":
            tx, r = dev(a["x"]), torch.zeros(1, dtype=torch.float64, device="cuda")
            args = U.upir_sum_args(tx.data_ptr(), U.UPIR_DT_F32, 0)
            lp = ctx.loop(U.UPIR_BODY_SUM, args, [(0, len(a["x"]), 1)], sched, H.make_red(U.UPIR_RED_SUM, r.data_ptr()))
            bufs.append((tx, r))
        else:
            tA, tx = dev(a["A"]), dev(a["x"])
            ty = torch.zeros(a["A"].shape[0], device="cuda")
            args = U.upir_matvec_args(tA.data_ptr(), tx.data_ptr(), ty.data_ptr(), 256, 256)
            lp = ctx.loop(U.UPIR_BODY_MATVEC, args, [(0, a["A"].shape[0], 1)], sched)
            bufs.append((tA, tx, ty))
        handles.append(lp)
    base = tok.data_ptr()
    for j in range(len(specs)):
        deps = [(base + 8 * j, U.UPIR_DEP_OUT)] + [(base + 8 * i, U.UPIR_DEP_IN) for i in preds[j]]
        assert ctx.task(handles[j], deps) == j
        assert ctx.task_preds(j) == preds[j]
    return handles, bufs, tok


def collect(specs, bufs):
    out = []
    for (kind, _), b in zip(specs, bufs):
        if kind == "axpy":
            out.append(b[1].cpu().numpy())
        elif kind == "sum":
            out.append(float(b[1].item()))
        else:
            out.append(b[2].cpu().numpy())
    return out


def check_against_oracle(specs, got):
    want = otasks.run_in_order(specs)
    for (kind, a), g, w in zip(specs, got, want):
        if kind == "axpy":
            assert np.array_equal(g, w["y"])
        elif kind == "sum":
            assert abs(g - w["s"]) <= 1e-5 * bodies.sum_abs_f64(a["x"])
        else:
            assert bodies.frob_rel(g.astype(np.float64), w["y"]) <= 1e-5


def stamps_ok(preds, start, done):
    for j, pj in enumerate(preds):
        for i in pj:
            assert done[i] < start[j], (i, j, done[i], start[j])
        assert start[j] <= done[j]


@pytest.mark.parametrize("mode", [U.UPIR_TASKWAIT_PLAIN, U.UPIR_TASKWAIT_BATCHED])
@pytest.mark.parametrize("seed,n,tile", [(1, 64, 0), (2, 200, 0), (3, 200, 4096), (4, 120, "static")])
def test_tasks_match_oracle(ctx, mode, seed, n, tile):
    note(f"tasks mode={mode} seed={seed} n={n} tile={tile}")
    specs, preds = make_workload(seed, n)
    handles, bufs, tok = build_tasks(ctx, specs, preds, tile)
    start = torch.zeros(n, dtype=torch.int64, device="cuda")
    done = torch.zeros(n, dtype=torch.int64, device="cuda")
    ctx.set_trace(tok.data_ptr(), start.data_ptr(), done.data_ptr())
    ctx.taskwait(mode)
    ctx.set_trace()
    got = collect(specs, bufs)
    check_against_oracle(specs, got)
    want_tok = otasks.tokens(preds)
    got_tok = [int(v) & (2 ** 64 - 1) for v in tok.cpu().numpy().tolist()]
    assert got_tok == want_tok
    stamps_ok(preds, start.cpu().numpy(), done.cpu().numpy())
    for h in handles:
        ctx.free(h)


def test_plain_and_batched_agree_bitwise(ctx):
    specs, preds = make_workload(4, 150)
    res = []
    for mode in (U.UPIR_TASKWAIT_PLAIN, U.UPIR_TASKWAIT_BATCHED):
        handles, bufs, tok = build_tasks(ctx, specs, preds)
        ctx.taskwait(mode)
        res.append(collect(specs, bufs))
        for h in handles:
            ctx.free(h)
    for (kind, _), a, b in zip(specs, res[0], res[1]):
        if kind != "sum":
            assert np.array_equal(a, b)


def test_batched_graph_replays(ctx):
    specs, preds = make_workload(5, 120, lmax=14)
    handles, bufs, tok = build_tasks(ctx, specs, preds)
    ctx.set_trace(tok.data_ptr())
    g = ctx.taskwait_graph(U.UPIR_TASKWAIT_BATCHED)
    ctx.set_trace()
    want_tok = otasks.tokens(preds)
    cur = [dict(a) for _, a in specs]
    for rep in range(3):
        tok.zero_()
        torch.cuda.synchronize()
        ctx.graph_launch(g)
        ctx.sync()
        # every replay applies each AXPY once more
        for j, (kind, a) in enumerate(specs):
            if kind == "axpy":
                cur[j]["y"] = bodies.axpy(2.5, a["x"], cur[j]["y"])
                assert np.array_equal(bufs[j][1].cpu().numpy(), cur[j]["y"])
        got_tok = [int(v) & (2 ** 64 - 1) for v in tok.cpu().numpy().tolist()]
        assert got_tok == want_tok
    ctx.graph_destroy(g)
    for h in handles:
        ctx.free(h)


def test_plain_graph_with_trace_replays(ctx):
    """The plain executor captured in a graph with the trace on: the
    predecessor lists reach the device before the capture and the graph owns
    them, so every replay writes the oracle's tokens and edge-ordered stamps."""
    specs, preds = make_workload(7, 90, lmax=13)
    handles, bufs, tok = build_tasks(ctx, specs, preds)
    n = len(specs)
    start = torch.zeros(n, dtype=torch.int64, device="cuda")
    done = torch.zeros(n, dtype=torch.int64, device="cuda")
    ctx.set_trace(tok.data_ptr(), start.data_ptr(), done.data_ptr())
    g = ctx.taskwait_graph(U.UPIR_TASKWAIT_PLAIN)
    ctx.set_trace()
    want_tok = otasks.tokens(preds)
    for rep in range(3):
        tok.zero_()
        ctx.graph_launch(g)
        ctx.sync()
        got_tok = [int(v) & (2 ** 64 - 1) for v in tok.cpu().numpy().tolist()]
        assert got_tok == want_tok, rep
        stamps_ok(preds, start.cpu().numpy(), done.cpu().numpy())
    ctx.graph_destroy(g)
    for h in handles:
        ctx.free(h)


@pytest.mark.parametrize("mode", [U.UPIR_TASKWAIT_PLAIN, U.UPIR_TASKWAIT_BATCHED])
def test_task_coverage(ctx, mode):
    n_tasks = 50
    lens = [int(v) for v in np.floor(2.0 ** (4 + 12 * synth.uniform01_f64(6, 0, n_tasks)))]
    cnts, handles = [], []
    for j, L in enumerate(lens):
        c = torch.zeros(L, dtype=torch.int32, device="cuda")
        lp = ctx.loop(U.UPIR_BODY_COVER, U.upir_cover_args(c.data_ptr()), [(0, L, 1)],
                      H.make_sched(U.UPIR_SCHED_AUTO, tile=(64,)))
        ctx.task(lp, [(0x1000, U.UPIR_DEP_INOUT)] if j % 3 == 0 else [])
        cnts.append(c)
        handles.append(lp)
    ctx.taskwait(mode)
    for c in cnts:
        assert (c.cpu().numpy() == 1).all()
    for h in handles:
        ctx.free(h)


def test_empty_taskwait(ctx):
    ctx.taskwait(U.UPIR_TASKWAIT_BATCHED)
    ctx.taskwait(U.UPIR_TASKWAIT_PLAIN)


# ------------------------------------------------------------- taskloop ----

MODES = [U.UPIR_TASKWAIT_PLAIN, U.UPIR_TASKWAIT_BATCHED]


@pytest.mark.parametrize("mode", MODES)
def test_taskloop_axpy_and_matvec(ctx, mode):
    """An AXPY cut by grainsize and a MATVEC cut by num_tasks: outputs equal
    the oracle's (AXPY bit-exact, MATVEC normwise 1e-5)."""
    note(f"taskloop axpy/matvec mode={mode}")
    n = 1_000_003
    x, y0 = synth.uniform_pm1(50, 0, n), synth.uniform_pm1(50, 1, n)
    tx, ty = dev(x), dev(y0)
    ax = ctx.loop(U.UPIR_BODY_AXPY, U.upir_axpy_args(2.5, 0, tx.data_ptr(), ty.data_ptr()), [(0, n, 1)])
    first, cnt = ctx.taskloop(ax, grainsize=65536)
    assert (first, cnt) == (0, otasks.taskloop_count(n, 65536))
    rows = 3001
    A, v = synth.uniform_pm1(51, 0, rows * 256).reshape(rows, 256), synth.uniform_pm1(51, 1, 256)
    tA, tv, tyv = dev(A), dev(v), torch.zeros(rows, device="cuda")
    mv = ctx.loop(U.UPIR_BODY_MATVEC, U.upir_matvec_args(tA.data_ptr(), tv.data_ptr(), tyv.data_ptr(), 256, 256),
                  [(0, rows, 1)])
    first2, cnt2 = ctx.taskloop(mv, num_tasks=7)
    assert (first2, cnt2) == (cnt, 7)
    ctx.taskwait(mode)
    assert np.array_equal(ty.cpu().numpy(), bodies.axpy(2.5, x, y0))
    assert bodies.frob_rel(tyv.cpu().numpy().astype(np.float64), bodies.matvec(A, v)) <= 1e-5
    ctx.free(ax)
    ctx.free(mv)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,lb,g,k", [(300007, 0, 0, 37), (100000, 5, 4096, 0), (10, 0, 0, 64)])
def test_taskloop_covers_each_iteration_once(ctx, mode, n, lb, g, k):
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    lp = ctx.loop(U.UPIR_BODY_COVER, U.upir_cover_args(cnt.data_ptr()), [(lb, lb + n, 1)])
    _, G = ctx.taskloop(lp, grainsize=g, num_tasks=k)
    assert G == otasks.taskloop_count(n, g, k)
    ctx.taskwait(mode)
    c = cnt.cpu().numpy()
    assert (c == 1).all(), int((c != 1).sum())
    ctx.free(lp)


@pytest.mark.parametrize("mode", MODES)
def test_taskloop_in_a_task_graph(ctx, mode):
    """task(out X) -> taskloop(in X, out Y) -> task(in Y): the taskloop's
    tasks run after the first task, side by side, and before the last; the
    token chain over the predecessors matches the oracle's graph."""
    note(f"taskloop graph mode={mode}")
    X, Y = 0x7000, 0x8000
    bufs = [(synth.uniform_pm1(52, 2 * i, 50000), synth.uniform_pm1(52, 2 * i + 1, 50000)) for i in range(3)]
    dbufs = [(dev(a), dev(b)) for a, b in bufs]
    lps = [ctx.loop(U.UPIR_BODY_AXPY, U.upir_axpy_args(2.5, 0, tx.data_ptr(), ty.data_ptr()), [(0, 50000, 1)])
           for tx, ty in dbufs]
    ctx.task(lps[0], [(X, U.UPIR_DEP_OUT)])
    first, G = ctx.taskloop(lps[1], num_tasks=5, deps=[(X, U.UPIR_DEP_IN), (Y, U.UPIR_DEP_OUT)])
    last = ctx.task(lps[2], [(Y, U.UPIR_DEP_IN)])
    assert (first, G, last) == (1, 5, 6)
    deps = [[(X, otasks.OUT)]] + [[(X, otasks.IN), (Y, otasks.OUT)]] * 5 + [[(Y, otasks.IN)]]
    want_preds = otasks.depend_edges(deps, [None] + [1] * 5 + [None])
    assert [ctx.task_preds(j) for j in range(7)] == want_preds
    tok = torch.zeros(7, dtype=torch.int64, device="cuda")
    ctx.set_trace(tok.data_ptr())
    ctx.taskwait(mode)
    ctx.set_trace()
    got = [int(v) & (2 ** 64 - 1) for v in tok.cpu().numpy().tolist()]
    assert got == otasks.tokens(want_preds)
    for (a, b), (_, ty) in zip(bufs, dbufs):
        assert np.array_equal(ty.cpu().numpy(), bodies.axpy(2.5, a, b))
    for lp in lps:
        ctx.free(lp)


# ------------------------------------------------ data_update as tasks ----

def _pipeline(ctx, x, y, chunks, X0, Y0, trace=None):
    """Per chunk: update(to) x_i, update(to) y_i, AXPY on the chunk,
    update(from) y_i; edges only within a chunk."""
    n = x.numel()
    Cn = n // chunks
    xp, yp = x.data_ptr(), y.data_ptr()
    lps = []
    for i in range(chunks):
        Xi, Yi = X0 + 64 * i, Y0 + 64 * i
        ctx.task_update(xp + 4 * i * Cn, 4 * Cn, U.UPIR_TO_DEVICE, [(Xi, U.UPIR_DEP_OUT)])
        ctx.task_update(yp + 4 * i * Cn, 4 * Cn, U.UPIR_TO_DEVICE, [(Yi, U.UPIR_DEP_OUT)])
        lp = ctx.loop(U.UPIR_BODY_AXPY, U.upir_axpy_args(2.5, 0, xp + 4 * i * Cn, yp + 4 * i * Cn), [(0, Cn, 1)],
                      None, None, device_ptrs=False)
        ctx.task(lp, [(Xi, U.UPIR_DEP_IN), (Yi, U.UPIR_DEP_INOUT)])
        ctx.task_update(yp + 4 * i * Cn, 4 * Cn, U.UPIR_FROM_DEVICE, [(Yi, U.UPIR_DEP_IN)])
        lps.append(lp)
    return lps


def test_update_tasks_pipeline_chunks(ctx):
    """Host (pinned) arrays mapped with alloc; copies in, AXPY and copies out
    as tasks over 8 chunks: the host result equals the oracle's AXPY and the
    token chain (task order across the three queues) equals the oracle's."""
    n, chunks = 1 << 22, 8
    x0, y0 = synth.uniform_pm1(53, 0, n), synth.uniform_pm1(53, 1, n)
    x = torch.from_numpy(x0).pin_memory()
    y = torch.from_numpy(y0).pin_memory()
    for t in (x, y):
        U.upir_data_map(ctx.h, t.data_ptr(), 4 * n, U.UPIR_MAP_ALLOC, U.UPIR_ACCESS_RW, None)
    lps = _pipeline(ctx, x, y, chunks, 0x10000, 0x20000)
    ntask = 4 * chunks
    deps = []
    for i in range(chunks):
        Xi, Yi = 0x10000 + 64 * i, 0x20000 + 64 * i
        deps += [[(Xi, otasks.OUT)], [(Yi, otasks.OUT)], [(Xi, otasks.IN), (Yi, otasks.INOUT)], [(Yi, otasks.IN)]]
    want_preds = otasks.depend_edges(deps)
    assert [ctx.task_preds(j) for j in range(ntask)] == want_preds
    tok = torch.zeros(ntask, dtype=torch.int64, device="cuda")
    ctx.set_trace(tok.data_ptr())
    y.zero_()  # the copies read y while the tasks run: reset the host value first
    y.copy_(torch.from_numpy(y0))
    ctx.taskwait(U.UPIR_TASKWAIT_PLAIN)
    ctx.set_trace()
    assert np.array_equal(y.numpy(), bodies.axpy(2.5, x0, y0))
    got = [int(v) & (2 ** 64 - 1) for v in tok.cpu().numpy().tolist()]
    assert got == otasks.tokens(want_preds)
    # untraced run (overlapping queues) gives the same result
    y.copy_(torch.from_numpy(y0))
    _pipeline(ctx, x, y, chunks, 0x10000, 0x20000)
    ctx.taskwait(U.UPIR_TASKWAIT_PLAIN)
    assert np.array_equal(y.numpy(), bodies.axpy(2.5, x0, y0))
    for t in (x, y):
        U.upir_data_unmap(ctx.h, t.data_ptr(), U.UPIR_MAP_ALLOC)
    for lp in lps:
        ctx.free(lp)


def test_update_tasks_rejected_where_unsupported(ctx):
    v = torch.zeros(1024).pin_memory()
    U.upir_data_map(ctx.h, v.data_ptr(), 4096, U.UPIR_MAP_ALLOC, U.UPIR_ACCESS_RW, None)
    ctx.task_update(v.data_ptr(), 0, U.UPIR_TO_DEVICE)
    assert U.raw("upir_taskwait")(ctx.h, U.UPIR_TASKWAIT_BATCHED) == U.UPIR_EUNSUPPORTED
    g = C.c_void_p()
    assert U.raw("upir_taskwait_graph")(ctx.h, U.UPIR_TASKWAIT_PLAIN, C.byref(g)) == U.UPIR_EUNSUPPORTED
    ctx.taskwait(U.UPIR_TASKWAIT_PLAIN)                       # still pending: runs now
    U.upir_data_unmap(ctx.h, v.data_ptr(), U.UPIR_MAP_ALLOC)
    w = np.zeros(16, np.float32)                              # never mapped
    ctx.task_update(w.ctypes.data, 64, U.UPIR_FROM_DEVICE)
    assert U.raw("upir_taskwait")(ctx.h, U.UPIR_TASKWAIT_PLAIN) == U.UPIR_ENOTMAPPED
