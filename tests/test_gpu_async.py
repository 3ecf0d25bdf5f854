"""GPU checks of deferred (async) reductions: arrive-compute at the end of
the loop kernel, wait-release at the next synchronisation point (sec. 5).

A loop whose reduction has ``async = 1`` leaves one partial per wavefront;
the fold runs in the next loop kernel on the context's stream (an extra
workgroup of a streaming loop or a Jacobi sweep, else workgroup 0 after its
own work), or as a one-workgroup kernel at
upir_sync / upir_reduce_wait / graph end / taskwait. Results must equal the synchronous path's: exact for max, min and
integer sums, within the float sum bound otherwise.
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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
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


def grid(h, w, seed):
    u = synth.uniform_01(seed, 0, h * w).reshape(h, w)
    u[0, :] = u[-1, :] = 0
    u[:, 0] = u[:, -1] = 0
    return u


def jacobi_handles(ctx, a, b, res, sweeps, sched=None, op=U.UPIR_RED_MAX):
    W = a.shape[1]
    hs = []
    for k in range(sweeps):
        src, dst = (a, b) if k % 2 == 0 else (b, a)
        args = U.upir_jacobi5_args(src.data_ptr(), dst.data_ptr(), W)
        red = H.make_red(op, res[k:].data_ptr(), init=float("inf") if op == U.UPIR_RED_MIN else 0.0, async_=True)
        hs.append(ctx.loop(U.UPIR_BODY_JACOBI5, args, [(1, a.shape[0] - 1, 1), (1, W - 1, 1)], sched, red))
    return hs


@pytest.mark.parametrize("shape,sched,op", [
    ((260, 1028), None, "max"),                                                   # tile kernel
    ((300, 516), H.make_sched(U.UPIR_SCHED_STATIC, tile=(16, 256)), "min"),
    ((130, 202), H.make_sched(U.UPIR_SCHED_STATIC), "max"),                       # generic kernel
    ((130, 202), H.make_sched(U.UPIR_SCHED_DYNAMIC, 3), "max"),                   # dynamic kernel
])
def test_async_jacobi_residuals_exact(ctx, shape, sched, op):
    note(f"async jacobi {shape} {op}")
    ops = {"max": U.UPIR_RED_MAX, "min": U.UPIR_RED_MIN}
    u0 = grid(*shape, seed=11)
    a, b = dev(u0), dev(u0)
    res = torch.full((5,), -1.0, dtype=torch.float64, device="cuda")
    hs = jacobi_handles(ctx, a, b, res, 5, sched, ops[op])
    ctx.launch(hs)
    ctx.sync()
    want_u, want_r = bodies.jacobi5(u0, 5, op=op)
    assert np.array_equal(b.cpu().numpy(), want_u)
    assert np.array_equal(res.cpu().numpy(), want_r)
    for h in hs:
        ctx.free(h)


def test_async_jacobi_graph_replays_with_eager_work_between(ctx):
    u0 = grid(516, 1032, seed=12)
    a, b = dev(u0), dev(u0)
    res = torch.zeros(10, dtype=torch.float64, device="cuda")
    hs = jacobi_handles(ctx, a, b, res, 10)
    ctx.launch(hs[:1])  # sizes scratch and fold buffers
    ctx.sync()
    ctx.graph_begin()
    ctx.launch(hs)
    g = ctx.graph_end()
    want_u, want_r = bodies.jacobi5(u0, 10)
    # an eager async loop left pending right before each replay
    x = dev(synth.uniform_pm1(13, 0, 50000))
    r2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    side = ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(x.data_ptr(), U.UPIR_DT_F32, 0), [(0, 50000, 1)], None,
                    H.make_red(U.UPIR_RED_MAX, r2.data_ptr(), init=-2.0, async_=True))
    for rep in range(3):
        a.copy_(dev(u0))
        b.copy_(dev(u0))
        res.zero_()
        r2.zero_()
        torch.cuda.synchronize()
        ctx.launch(side)
        ctx.graph_launch(g)
        ctx.sync()
        assert np.array_equal(a.cpu().numpy(), want_u), rep
        assert np.array_equal(res.cpu().numpy(), want_r), rep
        assert r2.item() == float(x.cpu().numpy().max()), rep
    ctx.graph_destroy(g)
    ctx.free(side)
    for h in hs:
        ctx.free(h)


def test_async_chain_then_matmul_and_sync(ctx):
    """Three async sums, each folded by the next kernel; a matmul (which
    cannot carry a fold) forces the standalone fold; integer sums exact."""
    n = 300007
    xs = [synth.uniform_pm1(14, i, n) for i in range(2)]
    ti = torch.arange(n, dtype=torch.int32, device="cuda")
    r = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
    ri = torch.zeros(1, dtype=torch.int64, device="cuda")
    txs = [dev(x) for x in xs]
    hs = [ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(txs[i].data_ptr(), U.UPIR_DT_F32, 0), [(0, n, 1)], None,
                   H.make_red(U.UPIR_RED_SUM, r[i:].data_ptr(), async_=True)) for i in range(2)]
    hs.append(ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(ti.data_ptr(), U.UPIR_DT_I32, 0), [(0, n, 1)], None,
                       H.make_red(U.UPIR_RED_SUM, ri.data_ptr(), init=5.0, async_=True)))
    M = 256
    A = synth.uniform_pm1(15, 0, M * M).reshape(M, M)
    tA, tC = dev(A), torch.zeros(M, M, device="cuda")
    mm = ctx.loop(U.UPIR_BODY_MATMUL_F32, U.upir_matmul_args(tA.data_ptr(), tA.data_ptr(), tC.data_ptr(), M, M, M, M,
                                                             None, 0), [(0, M, 1), (0, M, 1)])
    assert U.VARIANTS[ctx.resolve(mm)[2]] == "matmul_mfma"
    ctx.launch(hs + [mm])
    ctx.sync()
    got = r.cpu().numpy()
    for i in range(2):
        assert abs(got[i] - bodies.sum_f64(xs[i])) <= 1e-5 * bodies.sum_abs_f64(xs[i])
    assert int(ri.item()) == n * (n - 1) // 2 + 5
    assert got[2] == -1.0  # untouched
    assert bodies.frob_rel(tC.cpu().numpy(), bodies.matmul(A, A)) <= 1e-5
    for h in hs + [mm]:
        ctx.free(h)


def test_async_host_result_and_reduce_wait(ctx):
    v = synth.uniform_pm1(16, 0, 99991)
    t = dev(v)
    out = (C.c_double * 1)(-7.0)
    red = H.make_red(U.UPIR_RED_MIN, C.addressof(out), on_host=True, init=1.0, async_=True)
    lp = ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(t.data_ptr(), U.UPIR_DT_F32, 0), [(0, len(v), 1)], None, red)
    ctx.launch(lp)
    U.upir_reduce_wait(ctx.h, lp)
    assert out[0] == float(v.min())
    ctx.free(lp)


def test_async_then_free_before_sync(ctx):
    """Freeing the loop runs its pending fold first (the result survives)."""
    v = synth.uniform_pm1(17, 0, 4099)
    t = dev(v)
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    lp = ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(t.data_ptr(), U.UPIR_DT_F32, 0), [(0, len(v), 1)], None,
                  H.make_red(U.UPIR_RED_MAX, r.data_ptr(), async_=True))
    ctx.launch(lp)
    ctx.free(lp)
    torch.cuda.synchronize()
    assert r.item() == float(v.max())


def test_async_then_batched_tasks(ctx):
    v = synth.uniform_pm1(18, 0, 10007)
    t = dev(v)
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    lp = ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(t.data_ptr(), U.UPIR_DT_F32, 0), [(0, len(v), 1)], None,
                  H.make_red(U.UPIR_RED_MAX, r.data_ptr(), async_=True))
    ctx.launch(lp)
    nt = 6
    tok = torch.zeros(nt, dtype=torch.int64, device="cuda")
    preds = [[j - 1] if j else [] for j in range(nt)]
    ys, hs = [], []
    for j in range(nt):
        x = dev(synth.uniform_pm1(19, 2 * j, 3000))
        y0 = synth.uniform_pm1(19, 2 * j + 1, 3000)
        y = dev(y0)
        ys.append((x, y, y0))
        hs.append(ctx.loop(U.UPIR_BODY_AXPY, U.upir_axpy_args(2.5, 0, x.data_ptr(), y.data_ptr()), [(0, 3000, 1)]))
    base = tok.data_ptr()
    for j in range(nt):
        ctx.task(hs[j], [(base + 8 * j, U.UPIR_DEP_OUT)] + [(base + 8 * i, U.UPIR_DEP_IN) for i in preds[j]])
    ctx.set_trace(tok.data_ptr())
    ctx.taskwait(U.UPIR_TASKWAIT_BATCHED)
    ctx.set_trace()
    assert r.item() == float(v.max())
    for x, y, y0 in ys:
        assert np.array_equal(y.cpu().numpy(), bodies.axpy(2.5, x.cpu().numpy(), y0))
    got = [int(q) & (2 ** 64 - 1) for q in tok.cpu().numpy().tolist()]
    assert got == otasks.tokens(preds)
    for h in hs + [lp]:
        ctx.free(h)


def test_tuning_an_async_loop_leaves_its_result_alone(ctx):
    u0 = grid(260, 516, seed=20)
    a, b = dev(u0), dev(u0)
    res = torch.full((1,), -3.0, dtype=torch.float64, device="cuda")
    hs = jacobi_handles(ctx, a, b, res, 1)
    s_, p_, us = U.upir_sched(), U.upir_spmd(), C.c_double()
    U.upir_tune(ctx.h, None, hs[0], 2, C.byref(s_), C.byref(p_), C.byref(us))
    ctx.sync()
    assert res.item() == -3.0
    assert np.array_equal(b.cpu().numpy(), u0)
    ctx.launch(hs)
    ctx.sync()
    want_u, want_r = bodies.jacobi5(u0, 1)
    assert np.array_equal(b.cpu().numpy(), want_u) and res.item() == want_r[0]
    ctx.free(hs[0])


@pytest.mark.parametrize("jacobi_red", ["sync", "none", "async"])
def test_fold_rides_on_a_jacobi_sweep(ctx, jacobi_red):
    """An async loop's fold carried by the next kernel, a Jacobi sweep: by the
    sweep's extra workgroup, which is also the combiner when the sweep's own
    reduction is synchronous."""
    note(f"fold on jacobi ({jacobi_red})")
    v = synth.uniform_pm1(21, 0, 70001)
    t = dev(v)
    r1 = torch.zeros(1, dtype=torch.float64, device="cuda")
    first = ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(t.data_ptr(), U.UPIR_DT_F32, 0), [(0, len(v), 1)], None,
                     H.make_red(U.UPIR_RED_MAX, r1.data_ptr(), async_=True))
    u0 = grid(260, 1028, seed=22)
    a, b = dev(u0), dev(u0)
    r2 = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    red = None if jacobi_red == "none" else H.make_red(U.UPIR_RED_MAX, r2.data_ptr(), async_=(jacobi_red == "async"))
    sweep = ctx.loop(U.UPIR_BODY_JACOBI5, U.upir_jacobi5_args(a.data_ptr(), b.data_ptr(), u0.shape[1]),
                     [(1, u0.shape[0] - 1, 1), (1, u0.shape[1] - 1, 1)], None, red)
    assert U.VARIANTS[ctx.resolve(sweep)[2]] == "jacobi_tile"
    for rep in range(2):
        r1.zero_()
        r2.fill_(-1.0)
        ctx.launch([first, sweep])
        ctx.sync()
        assert r1.item() == float(v.max()), rep
        want_u, want_r = bodies.jacobi5(u0, 1)
        assert np.array_equal(b.cpu().numpy(), want_u), rep
        assert r2.item() == (-1.0 if jacobi_red == "none" else want_r[0]), rep
    ctx.free(first)
    ctx.free(sweep)


@pytest.mark.parametrize("stream_red", ["sync", "none", "async"])
@pytest.mark.parametrize("spmd", [None, (3, 64), (37, 256)])
def test_fold_rides_on_a_streaming_loop(ctx, stream_red, spmd):
    """An async loop's fold carried by the next kernel, an AXPY streaming loop:
    by one extra workgroup launched after the chunked ones, which is also the
    combiner when the AXPY loop's own sum is synchronous."""
    note(f"fold on axpy ({stream_red}, spmd {spmd})")
    v = synth.uniform_pm1(23, 0, 70001)
    t = dev(v)
    r1 = torch.zeros(1, dtype=torch.float64, device="cuda")
    first = ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(t.data_ptr(), U.UPIR_DT_F32, 0), [(0, len(v), 1)], None,
                     H.make_red(U.UPIR_RED_MAX, r1.data_ptr(), async_=True))
    n = 100003
    x, y0 = synth.uniform_pm1(24, 0, n), synth.uniform_pm1(24, 1, n)
    tx, ty = dev(x), dev(y0)
    r2 = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
    red = None if stream_red == "none" else H.make_red(U.UPIR_RED_SUM, r2.data_ptr(), async_=(stream_red == "async"))
    ax = ctx.loop(U.UPIR_BODY_AXPY, U.upir_axpy_args(2.5, 0, tx.data_ptr(), ty.data_ptr()), [(0, n, 1)], None, red)
    sp = H.make_spmd(*spmd) if spmd else None
    assert U.VARIANTS[ctx.resolve(ax, sp)[2]] == "stream4"
    want_y = bodies.axpy(2.5, x, y0)
    for rep in range(2):
        r1.zero_()
        r2.fill_(-7.0)
        ty.copy_(dev(y0))
        ctx.launch(first)
        ctx.launch(ax, sp)
        ctx.sync()
        assert r1.item() == float(v.max()), rep
        assert np.array_equal(ty.cpu().numpy(), want_y), rep
        if stream_red == "none":
            assert r2.item() == -7.0, rep
        else:
            assert abs(r2.item() - bodies.sum_f64(want_y)) <= 1e-5 * bodies.sum_abs_f64(want_y), rep
    ctx.free(first)
    ctx.free(ax)
