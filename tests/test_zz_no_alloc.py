"""upir_reduce_noalloc (the reduction that allocates nothing) against
upir_reduce and the oracle, through the C ABI.

For each case two calls run back to back, the second on a smaller input,
with nothing between them but stream order; each result must equal what
upir_reduce gives for the same input and launch (bit for bit: the same
kernels and plan), and the oracle's within the reduction tolerances (integer
exact, float max/min exact, float sums within 1e-5 * sum|x|). Integer and
float cases alternate, so each call must re-arm the shared scratch for its
own slot pattern. A captured graph of the call is replayed with eager work
between the replays; oversize launches and host results are refused.
"""
import ctypes as C
import math
import sys

import numpy as np
import pytest

import synth
from oracle import bodies
from oracle import reduce as oreduce
from paper_2209_10643_amd import helpers as H
from paper_2209_10643_amd import upir as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MAX_TEAMS = 4096  # UPIR_REDUCE_NOALLOC_MAX_TEAMS


def note(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    U.lib()
    s = torch.cuda.Stream()
    prev = torch.cuda.current_stream()
    torch.cuda.set_stream(s)
    c = H.Context(0, stream=s)
    yield c
    c.close()
    torch.cuda.set_stream(prev)


OPS = {U.UPIR_RED_SUM: "sum", U.UPIR_RED_MAX: "max", U.UPIR_RED_MIN: "min"}


def host_data(dtype, seed, stream, n):
    if dtype in (U.UPIR_DT_F32, U.UPIR_DT_F64):
        v = synth.uniform_pm1(seed, stream, n)
        return v if dtype == U.UPIR_DT_F32 else v.astype(np.float64)
    v = synth.int_range(seed, stream, n, -10 ** 6, 10 ** 6)
    return v.astype(np.int32 if dtype == U.UPIR_DT_I32 else np.int64)


def out_tensor(dtype, k):
    is_int = dtype in (U.UPIR_DT_I32, U.UPIR_DT_I64)
    return torch.zeros(k, dtype=torch.int64 if is_int else torch.float64, device="cuda")


def check_oracle(dtype, op, data, got):
    want = oreduce.reduce(OPS[op], data)
    if dtype in (U.UPIR_DT_I32, U.UPIR_DT_I64) or op != U.UPIR_RED_SUM:
        assert got == want, (got, want)
    else:
        assert abs(got - bodies.sum_f64(data)) <= 1e-5 * bodies.sum_abs_f64(data), (got, want)


# (dtype, op, n1, n2, spmd (teams, units) or None, schedule policy, chunk)
CASES = [
    (U.UPIR_DT_F32, U.UPIR_RED_SUM, 2 ** 22 + 3, 100003, None, U.UPIR_SCHED_AUTO, 0),
    (U.UPIR_DT_I64, U.UPIR_RED_SUM, 1000003, 4099, None, U.UPIR_SCHED_AUTO, 0),
    (U.UPIR_DT_F32, U.UPIR_RED_MAX, 777777, 65, (300, 256), U.UPIR_SCHED_STATIC, 0),
    (U.UPIR_DT_I32, U.UPIR_RED_MIN, 500001, 1, (37, 100), U.UPIR_SCHED_STATIC_CHUNK, 4),
    (U.UPIR_DT_F64, U.UPIR_RED_SUM, 300007, 2999, (64, 128), U.UPIR_SCHED_DYNAMIC, 64),
    (U.UPIR_DT_F32, U.UPIR_RED_MIN, 1 << 20, 0, (MAX_TEAMS, 64), U.UPIR_SCHED_STATIC, 0),
]


@pytest.mark.parametrize("case", CASES, ids=[f"c{i}" for i in range(len(CASES))])
def test_noalloc_matches_reduce_two_calls(ctx, case):
    dtype, op, n1, n2, spmd, pol, chunk = case
    note(f"no-alloc reduce: dtype={dtype} op={op} n1={n1} n2={n2} spmd={spmd} policy={pol}")
    init = 0.0 if op == U.UPIR_RED_SUM else (math.inf if op == U.UPIR_RED_MIN else -math.inf)
    if dtype in (U.UPIR_DT_I32, U.UPIR_DT_I64) and op != U.UPIR_RED_SUM:
        init = 2.0 ** 62 if op == U.UPIR_RED_MIN else -(2.0 ** 62)
    sp = C.byref(H.make_spmd(*spmd)) if spmd else None
    sc = C.byref(H.make_sched(pol, chunk))
    datas = [host_data(dtype, 41, 0, n1), host_data(dtype, 41, 1, n2)]
    devs = [torch.from_numpy(d).cuda() for d in datas]
    got = out_tensor(dtype, 2)
    ref = out_tensor(dtype, 2)
    # two no-alloc calls in a row, the second smaller; one synchronisation after both
    for k, t in enumerate(devs):
        red = H.make_red(op, got[k:].data_ptr(), init=init)
        U.upir_reduce_noalloc(ctx.h, op, dtype, t.data_ptr(), t.numel(), sp, sc, C.byref(red))
    ctx.sync()
    for k, t in enumerate(devs):
        red = H.make_red(op, ref[k:].data_ptr(), init=init)
        U.upir_reduce(ctx.h, op, dtype, t.data_ptr(), t.numel(), sp, sc, C.byref(red))
    ctx.sync()
    g, r = got.cpu().numpy(), ref.cpu().numpy()
    for k in range(2):
        assert g[k] == r[k] or (isinstance(g[k], float) and math.isnan(g[k]) and math.isnan(r[k])), (k, g[k], r[k])
        if datas[k].size == 0:
            assert g[k] == init
        else:
            check_oracle(dtype, op, datas[k], g[k].item())


def test_noalloc_refuses_oversize_and_host_results(ctx):
    t = torch.ones(1000, device="cuda")
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    f = U.raw("upir_reduce_noalloc")
    red = H.make_red(U.UPIR_RED_SUM, r.data_ptr())
    big = H.make_spmd(MAX_TEAMS + 1, 64)
    st = f(ctx.h, U.UPIR_RED_SUM, U.UPIR_DT_F32, t.data_ptr(), 1000, C.byref(big),
           C.byref(H.make_sched(U.UPIR_SCHED_STATIC)), C.byref(red))
    assert st == U.UPIR_EINVAL
    assert b"maximum" in U.lib().upir_last_error(ctx.h)
    res = (C.c_double * 1)()
    hred = H.make_red(U.UPIR_RED_SUM, C.addressof(res), on_host=True)
    assert f(ctx.h, U.UPIR_RED_SUM, U.UPIR_DT_F32, t.data_ptr(), 1000, None, None, C.byref(hred)) == U.UPIR_EINVAL
    ctx.sync()
    assert r.item() == 0.0  # nothing ran


def test_noalloc_graph_replays(ctx):
    """A graph captured around the call replays it correctly each time, with
    the data changed by eager work between replays."""
    n = 1 << 21
    x = torch.from_numpy(synth.uniform_pm1(42, 0, n)).cuda()
    r = torch.zeros(2, dtype=torch.float64, device="cuda")
    rr = torch.zeros(2, dtype=torch.float64, device="cuda")
    U.upir_graph_begin(ctx.h)
    try:
        red = H.make_red(U.UPIR_RED_SUM, r.data_ptr())
        U.upir_reduce_noalloc(ctx.h, U.UPIR_RED_SUM, U.UPIR_DT_F32, x.data_ptr(), n, None, None, C.byref(red))
        red = H.make_red(U.UPIR_RED_MAX, r[1:].data_ptr(), init=-math.inf)
        U.upir_reduce_noalloc(ctx.h, U.UPIR_RED_MAX, U.UPIR_DT_F32, x.data_ptr(), n, None, None, C.byref(red))
    finally:
        g = C.c_void_p()
        U.upir_graph_end(ctx.h, C.byref(g))
    for rep in range(4):
        x.copy_(torch.from_numpy(synth.uniform_pm1(42, 1 + rep, n)).cuda())
        ctx.sync()
        r.zero_()
        U.upir_graph_launch(ctx.h, g)
        ctx.sync()
        for k, op in enumerate((U.UPIR_RED_SUM, U.UPIR_RED_MAX)):
            red = H.make_red(op, rr[k:].data_ptr(), init=-math.inf if op == U.UPIR_RED_MAX else 0.0)
            U.upir_reduce(ctx.h, op, U.UPIR_DT_F32, x.data_ptr(), n, None, None, C.byref(red))
        ctx.sync()
        assert r.cpu().numpy().tolist() == rr.cpu().numpy().tolist(), rep
        xv = x.cpu().numpy()
        assert abs(r[0].item() - bodies.sum_f64(xv)) <= 1e-5 * bodies.sum_abs_f64(xv)
        assert r[1].item() == oreduce.reduce("max", xv)
    U.upir_graph_destroy(ctx.h, g)
