"""GPU parity of the worksharing loops against the CPU oracle.

Bit-exact: AXPY outputs, Jacobi grids and residuals, owner maps, coverage,
integer reductions, the BF16 split. Within tolerance: float sums
(|s - s_ref| <= 1e-5 * sum|y'|), matvec and float32 matmul (normwise 1e-5),
BF16 matmul (normwise 3e-3).
"""
import ctypes as C
import math
import sys

import numpy as np
import pytest

import synth
from oracle import bodies, loops as oloops
from oracle import reduce as oreduce
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


def dbl():
    return torch.zeros(1, dtype=torch.float64, device="cuda")


def run_axpy(ctx, x, y, a, dims, sched=None, spmd=None, red_op=U.UPIR_RED_SUM):
    tx, ty, r = dev(x), dev(y), dbl()
    args = U.upir_axpy_args(a, 0, tx.data_ptr(), ty.data_ptr())
    red = H.make_red(red_op, r.data_ptr()) if red_op else None
    lp = ctx.loop(U.UPIR_BODY_AXPY, args, dims, sched, red)
    variant = ctx.resolve(lp, spmd)[2]
    ctx.launch(lp, spmd)
    ctx.sync()
    out = ty.cpu().numpy(), float(r.item())
    ctx.free(lp)
    return out + (variant,)


AXPY_CASES = [
    (1, None, None), (63, None, None), (64, None, None), (65, None, None), (1000, None, None),
    (2 ** 20, None, None), (2 ** 20 + 3, None, None),
    (4099, H.make_sched(U.UPIR_SCHED_STATIC), H.make_spmd(7, 96)),
    (4099, H.make_sched(U.UPIR_SCHED_STATIC_CHUNK, 4), H.make_spmd(5, 128)),
    (4099, H.make_sched(U.UPIR_SCHED_STATIC_CHUNK, 3), H.make_spmd(3, 64)),
    (4096, H.make_sched(U.UPIR_SCHED_STATIC), H.make_spmd(4, 256)),
    (5000, H.make_sched(U.UPIR_SCHED_DYNAMIC, 2), H.make_spmd(9, 64)),
    (5000, H.make_sched(U.UPIR_SCHED_GUIDED, 1), H.make_spmd(9, 64)),
    (777, H.make_sched(U.UPIR_SCHED_STATIC, 0, U.UPIR_DIST_TEAMS), H.make_spmd(6, 32)),
    (777, H.make_sched(U.UPIR_SCHED_STATIC, 0, U.UPIR_DIST_UNITS), H.make_spmd(1, 100)),
]


@pytest.mark.parametrize("n,sched,spmd", AXPY_CASES)
def test_axpy_sum_parity(ctx, n, sched, spmd):
    note(f"axpy n={n}")
    x = synth.uniform_pm1(12345, 0, n)
    y = synth.uniform_pm1(12345, 1, n)
    got_y, got_s, variant = run_axpy(ctx, x, y, 2.5, [(0, n, 1)], sched, spmd)
    want_y = bodies.axpy(2.5, x, y)
    assert np.array_equal(got_y, want_y), f"variant {U.VARIANTS[variant]}"
    want_s = bodies.sum_f64(want_y)
    assert abs(got_s - want_s) <= 1e-5 * bodies.sum_abs_f64(want_y)


def test_stream_beyond_last_level_cache(ctx):
    """Large operands (>= 64 MiB) take the non-temporal streaming kernel:
    AXPY + sum at n = 40M + 3, SUM body at n = 70M + 1."""
    n = 40_000_003
    x, y = synth.uniform_pm1(21, 0, n), synth.uniform_pm1(21, 1, n)
    got_y, got_s, v = run_axpy(ctx, x, y, 2.5, [(0, n, 1)])
    assert U.VARIANTS[v] == "stream4"
    want_y = bodies.axpy(2.5, x, y)
    assert np.array_equal(got_y, want_y)
    assert abs(got_s - bodies.sum_f64(want_y)) <= 1e-5 * bodies.sum_abs_f64(want_y)
    del x, y, got_y, want_y
    m = 70_000_001
    z = synth.uniform_pm1(22, 0, m)
    tz, r = dev(z), dbl()
    lp = ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(tz.data_ptr(), U.UPIR_DT_F32, 0), [(0, m, 1)], None,
                  H.make_red(U.UPIR_RED_SUM, r.data_ptr()))
    assert U.VARIANTS[ctx.resolve(lp)[2]] == "stream4"
    ctx.launch(lp)
    ctx.sync()
    assert abs(r.item() - bodies.sum_f64(z)) <= 1e-5 * bodies.sum_abs_f64(z)
    ctx.free(lp)


def test_axpy_default_uses_vector_path(ctx):
    n = 2 ** 20
    x, y = synth.uniform_pm1(1, 0, n), synth.uniform_pm1(1, 1, n)
    _, _, variant = run_axpy(ctx, x, y, 2.5, [(0, n, 1)])
    assert U.VARIANTS[variant] == "stream4"


def test_axpy_strided_and_offset_loop(ctx):
    # for (i = 3; i < 1000; i += 7) and a descending loop: untouched entries stay
    n = 1000
    x, y = synth.uniform_pm1(2, 0, n), synth.uniform_pm1(2, 1, n)
    for dims in ([(3, 1000, 7)], [(999, -1, -5)]):
        got, s, _ = run_axpy(ctx, x, y, 2.5, dims, H.make_sched(U.UPIR_SCHED_STATIC), H.make_spmd(3, 64))
        idx = np.array([v for (v,) in oloops.serial_iterations(dims)])
        want = y.copy()
        want[idx] = bodies.axpy(2.5, x[idx], y[idx])
        assert np.array_equal(got, want)
        assert abs(s - bodies.sum_f64(want[idx])) <= 1e-5 * bodies.sum_abs_f64(want[idx])


def test_axpy_run_twice_deterministic(ctx):
    n = 300001
    x, y = synth.uniform_pm1(5, 0, n), synth.uniform_pm1(5, 1, n)
    a = run_axpy(ctx, x, y, 2.5, [(0, n, 1)])
    b = run_axpy(ctx, x, y, 2.5, [(0, n, 1)])
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


def test_empty_loop_reduction_gives_init(ctx):
    r = dbl()
    tx = torch.zeros(4, device="cuda")
    args = U.upir_sum_args(tx.data_ptr(), U.UPIR_DT_F32, 0)
    red = H.make_red(U.UPIR_RED_SUM, r.data_ptr(), init=1.5)
    lp = ctx.loop(U.UPIR_BODY_SUM, args, [(0, 0, 1)], None, red)
    ctx.launch(lp)
    ctx.sync()
    assert r.item() == 1.5
    ctx.free(lp)


@pytest.mark.parametrize("dtype,np_t", [(U.UPIR_DT_I32, np.int32), (U.UPIR_DT_I64, np.int64)])
def test_integer_reduce_closed_forms(ctx, dtype, np_t):
    for n in (0, 1, 64, 65, 100003, 2 ** 20 + 7):
        t = torch.arange(n, dtype=torch.int32 if np_t is np.int32 else torch.int64, device="cuda")
        res = (C.c_int64 * 1)()
        # init 0 is folded in once: max(0, n-1), min(0, 0); an empty loop gives init
        for op, want in ((U.UPIR_RED_SUM, n * (n - 1) // 2), (U.UPIR_RED_MAX, max(n - 1, 0)),
                         (U.UPIR_RED_MIN, 0)):
            red = H.make_red(op, C.addressof(res), on_host=True)
            U.upir_reduce(ctx.h, op, dtype, t.data_ptr(), n, None, None, C.byref(red))
            assert res[0] == want, (n, op)


def test_float_reduce_max_min_exact(ctx):
    v = synth.uniform_pm1(8, 0, 123457)
    t = dev(v)
    res = (C.c_double * 1)()
    for op, want in ((U.UPIR_RED_MAX, float(v.max())), (U.UPIR_RED_MIN, float(v.min()))):
        red = H.make_red(op, C.addressof(res), on_host=True)
        U.upir_reduce(ctx.h, op, U.UPIR_DT_F32, t.data_ptr(), len(v), None, None, C.byref(red))
        assert res[0] == want
    red = H.make_red(U.UPIR_RED_SUM, C.addressof(res), on_host=True)
    U.upir_reduce(ctx.h, U.UPIR_RED_SUM, U.UPIR_DT_F64, dev(v.astype(np.float64)).data_ptr(), len(v), None, None,
                  C.byref(red))
    assert abs(res[0] - bodies.sum_f64(v)) <= 1e-12 * bodies.sum_abs_f64(v)


# A team of U units with U % 64 != 0 ends in a partial wavefront (or is one,
# for U < 64). Lanes past the end do not exist: the wavefront reduction must
# take the op's identity for them, never 0 or an undefined register. MIN
# over positive data and MAX over negative data see a wrong 0 at once; init
# is the op's identity so the data alone decide the result.
PARTIAL_UNITS = [32, 96, 100]


@pytest.mark.parametrize("units", PARTIAL_UNITS)
@pytest.mark.parametrize("pol", [U.UPIR_SCHED_STATIC, U.UPIR_SCHED_STATIC_CHUNK])
def test_partial_wavefront_float_min_max(ctx, units, pol):
    note(f"partial wavefront float units={units} pol={pol}")
    n = 10007
    pos = synth.uniform_01(31, 0, n) + np.float32(0.5)   # all in [0.5, 1.5)
    neg = -pos
    sched = H.make_sched(pol, 4 if pol == U.UPIR_SCHED_STATIC_CHUNK else 0)
    spmd = H.make_spmd(7, units)
    for data, op, init, want in ((pos, U.UPIR_RED_MIN, math.inf, float(pos.min())),
                                 (neg, U.UPIR_RED_MAX, -math.inf, float(neg.max()))):
        t, r = dev(data), dbl()
        red = H.make_red(op, r.data_ptr(), init=init)
        lp = ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(t.data_ptr(), U.UPIR_DT_F32, 0), [(0, n, 1)], sched, red)
        ctx.launch(lp, spmd)
        ctx.sync()
        ctx.free(lp)
        assert r.item() == want == oreduce.reduce("min" if op == U.UPIR_RED_MIN else "max", data), (units, op)
    # AXPY loop reducing its outputs y' (all positive: a x + y with x, y >= 0.5)
    x, y = pos, synth.uniform_01(31, 1, n) + np.float32(0.5)
    tx, ty, r = dev(x), dev(y), dbl()
    lp = ctx.loop(U.UPIR_BODY_AXPY, U.upir_axpy_args(2.5, 0, tx.data_ptr(), ty.data_ptr()), [(0, n, 1)], sched,
                  H.make_red(U.UPIR_RED_MIN, r.data_ptr(), init=math.inf))
    ctx.launch(lp, spmd)
    ctx.sync()
    ctx.free(lp)
    want = bodies.axpy(2.5, x, y)
    assert np.array_equal(ty.cpu().numpy(), want)
    assert r.item() == oreduce.reduce("min", want)


@pytest.mark.parametrize("units", PARTIAL_UNITS)
def test_partial_wavefront_int64_min_max(ctx, units):
    note(f"partial wavefront int64 units={units}")
    n = 5003
    v = synth.int_range(32, 0, n, 1000, 10 ** 9).astype(np.int64)
    res = (C.c_int64 * 1)()
    spmd = H.make_spmd(5, units)
    for data, op, init in ((v, U.UPIR_RED_MIN, 2.0 ** 62), (-v, U.UPIR_RED_MAX, -(2.0 ** 62))):
        t = dev(data)
        red = H.make_red(op, C.addressof(res), on_host=True, init=init)
        U.upir_reduce(ctx.h, op, U.UPIR_DT_I64, t.data_ptr(), n, C.byref(spmd),
                      C.byref(H.make_sched(U.UPIR_SCHED_STATIC)), C.byref(red))
        want = oreduce.reduce("min" if op == U.UPIR_RED_MIN else "max", data)
        assert res[0] == want, (units, op, res[0], want)


@pytest.mark.parametrize("units", PARTIAL_UNITS)
def test_partial_wavefront_jacobi_min_residual(ctx, units):
    """Jacobi residual MIN through the generic kernel with partial wavefronts:
    on a field with no fixed point in the interior every |u1 - u0| is > 0."""
    note(f"partial wavefront jacobi units={units}")
    N = 67
    u = synth.uniform_01(33, 0, N * N).reshape(N, N) + np.float32(1.0)
    u[0, :] = u[-1, :] = 0
    u[:, 0] = u[:, -1] = 0
    a, b, r = dev(u), dev(u), dbl()
    red = H.make_red(U.UPIR_RED_MIN, r.data_ptr(), init=math.inf)
    lp = ctx.loop(U.UPIR_BODY_JACOBI5, U.upir_jacobi5_args(a.data_ptr(), b.data_ptr(), N),
                  [(1, N - 1, 1), (1, N - 1, 1)], H.make_sched(U.UPIR_SCHED_STATIC), red)
    ctx.launch(lp, H.make_spmd(9, units))
    ctx.sync()
    ctx.free(lp)
    wu, wr = bodies.jacobi5(u, 1, op="min")
    assert np.array_equal(b.cpu().numpy(), wu)
    assert r.item() == wr[0] and wr[0] > 0


# ----------------------------------------------------------- owner maps ----

def run_owner(ctx, dims, sched, spmd):
    n = int(np.prod([oloops.trip_count(*d) for d in dims]))
    out = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    args = U.upir_owner_args(out.data_ptr())
    lp = ctx.loop(U.UPIR_BODY_OWNER, args, dims, sched)
    sp, _, _ = ctx.resolve(lp, spmd)
    ctx.launch(lp, spmd)
    ctx.sync()
    ctx.free(lp)
    return out.cpu().numpy()[:n].astype(np.int64), sp.num_teams, sp.num_units


OWNER_CASES = [
    ([(0, 1000, 1)], U.UPIR_SCHED_STATIC, 0, U.UPIR_DIST_TEAMS_UNITS, 7, 64, None),
    ([(0, 1000, 1)], U.UPIR_SCHED_STATIC, 0, U.UPIR_DIST_TEAMS_UNITS, 9, 130, None),
    ([(5, 300, 3)], U.UPIR_SCHED_STATIC_CHUNK, 17, U.UPIR_DIST_TEAMS_UNITS, 3, 64, None),
    ([(0, 4099, 1)], U.UPIR_SCHED_STATIC_CHUNK, 4, U.UPIR_DIST_TEAMS_UNITS, 5, 128, None),
    ([(0, 500, 1)], U.UPIR_SCHED_STATIC, 0, U.UPIR_DIST_TEAMS, 6, 64, None),
    ([(0, 500, 1)], U.UPIR_SCHED_STATIC_CHUNK, 3, U.UPIR_DIST_TEAMS, 6, 64, None),
    ([(0, 500, 1)], U.UPIR_SCHED_STATIC, 0, U.UPIR_DIST_UNITS, 1, 96, None),
    ([(0, 500, 1)], U.UPIR_SCHED_STATIC_CHUNK, 2, U.UPIR_DIST_UNITS, 1, 96, None),
    ([(0, 37, 1), (3, 50, 2)], U.UPIR_SCHED_STATIC, 0, U.UPIR_DIST_TEAMS_UNITS, 4, 64, None),
    ([(9, 0, -2), (1, 7, 1), (4, -4, -3)], U.UPIR_SCHED_STATIC_CHUNK, 2, U.UPIR_DIST_TEAMS_UNITS, 3, 64, None),
    ([(1, 70, 1), (1, 133, 1)], U.UPIR_SCHED_STATIC, 0, U.UPIR_DIST_TEAMS_UNITS, 5, 64, (16, 32)),
    ([(0, 33, 1), (2, 40, 1)], U.UPIR_SCHED_STATIC_CHUNK, 2, U.UPIR_DIST_TEAMS_UNITS, 3, 96, (8, 8)),
    ([(0, 9, 1), (1, 10, 1), (0, 13, 1)], U.UPIR_SCHED_STATIC, 0, U.UPIR_DIST_TEAMS_UNITS, 4, 64, (2, 4, 4)),
]


@pytest.mark.parametrize("dims,pol,chunk,dist,T,Uu,tile", OWNER_CASES)
def test_owner_map_matches_oracle(ctx, dims, pol, chunk, dist, T, Uu, tile):
    note(f"owner {dims} pol={pol} chunk={chunk} dist={dist} T={T} U={Uu} tile={tile}")
    sched = H.make_sched(pol, chunk, dist, tile or (0, 0, 0))
    got, t_, u_ = run_owner(ctx, dims, sched, H.make_spmd(T, Uu))
    assert (t_, u_) == (T, Uu)
    n = len(got)
    oname = {U.UPIR_SCHED_STATIC: oloops.STATIC, U.UPIR_SCHED_STATIC_CHUNK: oloops.STATIC_CHUNK}[pol]
    if tile:
        team, unit = oloops.tiled_owner_map(dims, tile, T, Uu, oname, chunk)
    else:
        dname = {U.UPIR_DIST_TEAMS_UNITS: oloops.TEAMS_UNITS, U.UPIR_DIST_TEAMS: oloops.TEAMS,
                 U.UPIR_DIST_UNITS: oloops.UNITS}[dist]
        team, unit = oloops.owner_map(n, T, Uu, oname, chunk, dname)
    assert np.array_equal(got, team * Uu + unit)


@pytest.mark.parametrize("pol,chunk,T,Uu", [
    (U.UPIR_SCHED_DYNAMIC, 1, 13, 64), (U.UPIR_SCHED_DYNAMIC, 7, 64, 256), (U.UPIR_SCHED_GUIDED, 1, 13, 64),
    (U.UPIR_SCHED_GUIDED, 5, 200, 128), (U.UPIR_SCHED_STATIC_CHUNK, 4, 0, 0), (U.UPIR_SCHED_STATIC, 0, 11, 96),
])
def test_coverage_each_iteration_once(ctx, pol, chunk, T, Uu):
    n = 100003
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    args = U.upir_cover_args(cnt.data_ptr())
    lp = ctx.loop(U.UPIR_BODY_COVER, args, [(0, n, 1)], H.make_sched(pol, chunk))
    sp = H.make_spmd(T, Uu)
    for rep in range(3):  # the dynamic counter re-arms itself
        ctx.launch(lp, sp)
        ctx.sync()
        c = cnt.cpu().numpy()
        assert (c == rep + 1).all(), (rep, int((c != rep + 1).sum()))
    ctx.free(lp)


# --------------------------------------------------------------- Jacobi ----

def jacobi_grid(H_, W, seed=7):
    u = synth.uniform_01(seed, 0, H_ * W).reshape(H_, W)
    u[0, :] = u[-1, :] = 0
    u[:, 0] = u[:, -1] = 0
    return u


def run_jacobi(ctx, u0, sweeps, sched, spmd=None, graph=False, replays=1, op=None):
    Hh, W = u0.shape
    a, b = dev(u0), dev(u0)
    res = torch.zeros(sweeps, dtype=torch.float64, device="cuda")
    dims = [(1, Hh - 1, 1), (1, W - 1, 1)]
    handles = []
    for k in range(sweeps):
        src, dst = (a, b) if k % 2 == 0 else (b, a)
        args = U.upir_jacobi5_args(src.data_ptr(), dst.data_ptr(), W)
        op_ = U.UPIR_RED_MAX if op is None else op
        red = H.make_red(op_, res[k:].data_ptr(), init=float("inf") if op_ == U.UPIR_RED_MIN else 0.0)
        handles.append(ctx.loop(U.UPIR_BODY_JACOBI5, args, dims, sched, red))
    variant = ctx.resolve(handles[0], spmd)[2]
    outs = []
    if graph:
        ctx.launch(handles[:1], spmd)  # sizes the scratch before capture
        ctx.sync()
        a.copy_(dev(u0))
        b.copy_(dev(u0))
        ctx.graph_begin()
        ctx.launch(handles, spmd)
        g = ctx.graph_end()
        for _ in range(replays):
            a.copy_(dev(u0))
            b.copy_(dev(u0))
            res.zero_()
            torch.cuda.synchronize()
            ctx.graph_launch(g)
            ctx.sync()
            fin = (a if sweeps % 2 == 0 else b).cpu().numpy()
            outs.append((fin, res.cpu().numpy()))
        ctx.graph_destroy(g)
    else:
        ctx.launch(handles, spmd)
        ctx.sync()
        fin = (a if sweeps % 2 == 0 else b).cpu().numpy()
        outs.append((fin, res.cpu().numpy()))
    for h in handles:
        ctx.free(h)
    return outs, variant


JACOBI_CASES = [
    ((5, 7), None, None, "generic"),
    ((3, 4), None, None, "jacobi_tile"),                   # one interior row of two points
    ((3, 1028), None, None, "jacobi_tile"),                # one interior row
    ((1000, 4), None, None, "jacobi_tile"),                # a thin column
    ((33, 65), None, None, "generic"),                     # ld % 4 != 0 -> generic path
    ((64, 64), None, None, "jacobi_tile"),
    ((260, 1028), None, None, "jacobi_tile"),              # ragged tiles in both directions
    ((300, 516), H.make_sched(U.UPIR_SCHED_STATIC, tile=(8, 256)), H.make_spmd(7, 128), "jacobi_tile"),
    ((300, 516), H.make_sched(U.UPIR_SCHED_STATIC_CHUNK, 3, tile=(32, 256)), H.make_spmd(5, 512), "jacobi_tile"),
    ((130, 200), H.make_sched(U.UPIR_SCHED_STATIC), H.make_spmd(11, 64), "generic"),
    ((130, 200), H.make_sched(U.UPIR_SCHED_STATIC_CHUNK, 5, tile=(4, 16)), H.make_spmd(3, 64), "generic"),
    ((130, 200), H.make_sched(U.UPIR_SCHED_DYNAMIC, 3), H.make_spmd(17, 64), "dynamic"),
]


@pytest.mark.parametrize("shape,sched,spmd,variant", JACOBI_CASES)
def test_jacobi_parity(ctx, shape, sched, spmd, variant):
    note(f"jacobi {shape} variant {variant}")
    u0 = jacobi_grid(*shape)
    outs, v = run_jacobi(ctx, u0, 6, sched, spmd)
    assert U.VARIANTS[v] == variant
    want_u, want_r = bodies.jacobi5(u0, 6)
    got_u, got_r = outs[0]
    assert np.array_equal(got_u, want_u)
    assert np.array_equal(got_r, want_r)


OPS = {"max": U.UPIR_RED_MAX, "min": U.UPIR_RED_MIN, "sum": U.UPIR_RED_SUM}


@pytest.mark.parametrize("th,units,op", [
    (4, 64, "max"), (16, 192, "max"), (64, 64, "max"), (64, 512, "min"), (8, 256, "sum"), (32, 128, "sum"),
    (32, 256, "min"), (128, 256, "max"), (128, 1024, "sum"),
])
def test_jacobi_tile_strips_and_ops(ctx, th, units, op):
    """Tile heights, wavefront counts (192: strips of unequal length) and the
    three residual reductions on a grid with ragged tiles on all sides."""
    note(f"jacobi tile ({th}, 256) units {units} op {op}")
    u0 = jacobi_grid(203, 780, seed=th + units)
    sched = H.make_sched(U.UPIR_SCHED_STATIC, tile=(th, 256))
    outs, v = run_jacobi(ctx, u0, 3, sched, H.make_spmd(0, units), op=OPS[op])
    assert U.VARIANTS[v] == "jacobi_tile"
    want_u, want_r = bodies.jacobi5(u0, 3, op=op)
    got_u, got_r = outs[0]
    assert np.array_equal(got_u, want_u)
    if op == "sum":
        # float64 sum of n non-negative terms in another order: |error| <= n 2^-53 sum
        n = (u0.shape[0] - 2) * (u0.shape[1] - 2)
        assert np.all(np.abs(got_r - want_r) <= n * 2.0 ** -53 * want_r)
    else:
        assert np.array_equal(got_r, want_r)


@pytest.mark.parametrize("box,th,units,op", [
    (((5, 203), (3, 517)), 16, 256, "max"),    # box edges inside lanes on both sides
    (((1, 209), (2, 518)), 64, 512, "min"),
    (((7, 150), (1, 513)), 8, 64, "sum"),      # left edge on a lane boundary, right edge inside a lane
    (((2, 3), (255, 258)), 4, 128, "max"),     # one row across a tile boundary
])
def test_jacobi_tile_sub_box(ctx, box, th, units, op):
    """A loop box strictly inside the grid: only box points are written (the
    rest of the destination keeps its sentinel), lanes whose four columns
    straddle a box edge load and store column by column, and the residual
    covers the box alone."""
    (i0, i1), (j0, j1) = box
    note(f"jacobi sub-box {box} tile ({th}, 256) units {units} op {op}")
    u0 = jacobi_grid(210, 532, seed=31 + th)
    src = dev(u0)
    dst = torch.full(u0.shape, -7.0, device="cuda")
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    op_ = OPS[op]
    red = H.make_red(op_, res.data_ptr(), init=float("inf") if op_ == U.UPIR_RED_MIN else 0.0)
    lp = ctx.loop(U.UPIR_BODY_JACOBI5, U.upir_jacobi5_args(src.data_ptr(), dst.data_ptr(), u0.shape[1]),
                  [(i0, i1, 1), (j0, j1, 1)], H.make_sched(U.UPIR_SCHED_STATIC, tile=(th, 256)), red)
    sp = H.make_spmd(0, units)
    assert U.VARIANTS[ctx.resolve(lp, sp)[2]] == "jacobi_tile"
    ctx.launch(lp, sp)
    ctx.sync()
    ctx.free(lp)
    full = bodies.jacobi5_sweep_f32(u0)
    want = np.full(u0.shape, -7.0, np.float32)
    want[i0:i1, j0:j1] = full[i0:i1, j0:j1]
    assert np.array_equal(dst.cpu().numpy(), want)
    # the oracle's residual over the interior of the box grown by its halo
    want_r = bodies.update_f64(full[i0 - 1:i1 + 1, j0 - 1:j1 + 1], u0[i0 - 1:i1 + 1, j0 - 1:j1 + 1], op)
    got_r = res.item()
    if op == "sum":
        n = (i1 - i0) * (j1 - j0)
        assert abs(got_r - want_r) <= n * 2.0 ** -53 * want_r
    else:
        assert got_r == want_r


def test_jacobi_linear_field_is_fixed(ctx):
    N = 300
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    u = ((i + 2 * j) * 2.0 ** -10).astype(np.float32)
    outs, _ = run_jacobi(ctx, u, 4, None)
    assert np.array_equal(outs[0][0], u) and (outs[0][1] == 0).all()


def test_jacobi_graph_replays(ctx):
    u0 = jacobi_grid(516, 1032, seed=9)
    outs, v = run_jacobi(ctx, u0, 10, None, graph=True, replays=3)
    want_u, want_r = bodies.jacobi5(u0, 10)
    for got_u, got_r in outs:
        assert np.array_equal(got_u, want_u)
        assert np.array_equal(got_r, want_r)


def test_graph_replay_after_scratch_growth(ctx):
    """A graph captured with T teams keeps working after an eager launch of
    the same loop with more teams than its reduction scratch held (the
    scratch grows; the block the graph addresses must stay alive)."""
    n = 1 << 20
    x = synth.uniform_pm1(41, 0, n)
    t, r = dev(x), dbl()
    lp = ctx.loop(U.UPIR_BODY_SUM, U.upir_sum_args(t.data_ptr(), U.UPIR_DT_F32, 0), [(0, n, 1)],
                  H.make_sched(U.UPIR_SCHED_STATIC), H.make_red(U.UPIR_RED_SUM, r.data_ptr()))
    want, tol = bodies.sum_f64(x), 1e-5 * bodies.sum_abs_f64(x)
    small, big = H.make_spmd(100, 256), H.make_spmd(9000, 64)
    ctx.launch(lp, small)  # eager first, so nothing has to grow during capture
    ctx.sync()
    ctx.graph_begin()
    ctx.launch(lp, small)
    g = ctx.graph_end()
    for k in range(3):
        r.zero_()
        ctx.launch(lp, big)  # 9000 workgroups: more slots than the capture's block
        ctx.sync()
        assert abs(r.item() - want) <= tol, ("eager", k)
        r.zero_()
        ctx.graph_launch(g)
        ctx.sync()
        assert abs(r.item() - want) <= tol, ("replay", k)
    ctx.graph_destroy(g)
    ctx.free(lp)


# --------------------------------------------------------------- matvec ----

@pytest.mark.parametrize("rows,cols,sched,spmd", [
    (1000, 256, None, None), (37, 100, None, None), (513, 300, None, None),
    (1000, 256, H.make_sched(U.UPIR_SCHED_STATIC), H.make_spmd(5, 128)),
    (999, 256, H.make_sched(U.UPIR_SCHED_STATIC_CHUNK, 3), H.make_spmd(7, 256)),
    # rows of at least four 256-column blocks: eight / four blocks per trip, then one at a time
    (300, 1024, None, None), (129, 2316, None, None), (64, 4096, None, None), (33, 3003, None, None),
    (70, 2560, H.make_sched(U.UPIR_SCHED_STATIC), H.make_spmd(3, 128)),
])
def test_matvec_parity(ctx, rows, cols, sched, spmd):
    A = synth.uniform_pm1(11, 0, rows * cols).reshape(rows, cols)
    x = synth.uniform_pm1(11, 1, cols)
    tA, tx = dev(A), dev(x)
    ty = torch.zeros(rows, device="cuda")
    r = dbl()
    args = U.upir_matvec_args(tA.data_ptr(), tx.data_ptr(), ty.data_ptr(), cols, cols)
    lp = ctx.loop(U.UPIR_BODY_MATVEC, args, [(0, rows, 1)], sched, H.make_red(U.UPIR_RED_SUM, r.data_ptr()))
    ctx.launch(lp, spmd)
    ctx.sync()
    got = ty.cpu().numpy().astype(np.float64)
    want = bodies.matvec(A, x)
    assert bodies.frob_rel(got, want) <= 1e-5
    for rr in (0, rows // 2, rows - 1):
        assert abs(got[rr] - bodies.matvec_row(A[rr], x)) <= 1e-5 * np.abs(A[rr] * x).sum() + 1e-30
    assert abs(r.item() - got.sum()) <= 1e-5 * np.abs(got).sum()
    ctx.free(lp)


def test_matvec_schedules_bitwise_equal(ctx):
    rows, cols = 777, 256
    A = synth.uniform_pm1(12, 0, rows * cols).reshape(rows, cols)
    x = synth.uniform_pm1(12, 1, cols)
    tA, tx = dev(A), dev(x)
    outs = []
    for sched, sp in ((None, None), (H.make_sched(U.UPIR_SCHED_STATIC), H.make_spmd(3, 64))):
        ty = torch.zeros(rows, device="cuda")
        args = U.upir_matvec_args(tA.data_ptr(), tx.data_ptr(), ty.data_ptr(), cols, cols)
        lp = ctx.loop(U.UPIR_BODY_MATVEC, args, [(0, rows, 1)], sched)
        ctx.launch(lp, sp)
        ctx.sync()
        outs.append(ty.cpu().numpy())
        ctx.free(lp)
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("cols", [2316, 4096])
def test_matvec_wide_rows_loop_and_engine_bitwise(ctx, cols):
    """Rows of many 256-column blocks: the loop kernel (blocks loaded eight or
    four at a time) and the batched engine (one block at a time) add the same
    products in the same order, so their outputs are identical bits."""
    rows = 200
    A = synth.uniform_pm1(13, 0, rows * cols).reshape(rows, cols)
    x = synth.uniform_pm1(13, 1, cols)
    tA, tx = dev(A), dev(x)
    outs = []
    for mode in ("loop", "engine"):
        ty = torch.zeros(rows, device="cuda")
        args = U.upir_matvec_args(tA.data_ptr(), tx.data_ptr(), ty.data_ptr(), cols, cols)
        lp = ctx.loop(U.UPIR_BODY_MATVEC, args, [(0, rows, 1)], None)
        if mode == "loop":
            ctx.launch(lp)
        else:
            ctx.task(lp)
            ctx.taskwait(U.UPIR_TASKWAIT_BATCHED)
        ctx.sync()
        outs.append(ty.cpu().numpy())
        ctx.free(lp)
    assert np.array_equal(outs[0], outs[1])
    assert bodies.frob_rel(outs[0].astype(np.float64), bodies.matvec(A, x)) <= 1e-5


# ---------------------------------------------------------- data mapping ----

def test_mapped_axpy_host_pointers(ctx):
    n = 10007
    x = synth.uniform_pm1(3, 0, n)
    y = synth.uniform_pm1(3, 1, n)
    want = bodies.axpy(2.5, x, y)
    xp, yp = x.ctypes.data, y.ctypes.data
    U.upir_data_map(ctx.h, xp, x.nbytes, U.UPIR_MAP_TO, U.UPIR_ACCESS_RO, None)
    U.upir_data_map(ctx.h, yp, y.nbytes, U.UPIR_MAP_TOFROM, U.UPIR_ACCESS_RW, None)
    res = (C.c_double * 1)()
    args = U.upir_axpy_args(2.5, 0, xp, yp)
    red = H.make_red(U.UPIR_RED_SUM, C.addressof(res), on_host=True, async_=True)
    lp = ctx.loop(U.UPIR_BODY_AXPY, args, [(0, n, 1)], None, red, device_ptrs=False)
    ctx.launch(lp)
    U.upir_reduce_wait(ctx.h, lp)                    # wait-release step
    assert abs(res[0] - bodies.sum_f64(want)) <= 1e-5 * bodies.sum_abs_f64(want)
    # explicit update brings y back while it stays mapped
    y2 = np.zeros_like(y)
    U.upir_data_update(ctx.h, yp, 0, U.UPIR_FROM_DEVICE)
    y2[:] = y
    assert np.array_equal(y2, want)
    U.upir_data_unmap(ctx.h, xp, U.UPIR_MAP_TO)
    y[:] = 0
    U.upir_data_unmap(ctx.h, yp, U.UPIR_MAP_TOFROM)   # copies back on the last unmap
    assert np.array_equal(y, want)
    # the body now refers to unmapped memory
    arr = (C.c_void_p * 1)(lp.value)
    assert U.raw("upir_spmd_launch")(ctx.h, None, arr, 1) == U.UPIR_ENOTMAPPED
    ctx.free(lp)


def test_map_refcount_and_update_to(ctx):
    v = np.arange(1024, dtype=np.float32)
    p = v.ctypes.data
    U.upir_data_map(ctx.h, p, v.nbytes, U.UPIR_MAP_TO, U.UPIR_ACCESS_RW, None)
    U.upir_data_map(ctx.h, p, v.nbytes, U.UPIR_MAP_TOFROM, U.UPIR_ACCESS_RW, None)   # present: no copy
    v[:] = -1
    U.upir_data_update(ctx.h, p + 64, 64, U.UPIR_TO_DEVICE)                         # elements 16..31
    U.upir_data_unmap(ctx.h, p, U.UPIR_MAP_FROM)                                    # ref 2 -> 1: no copy
    assert (v == -1).all()
    U.upir_data_unmap(ctx.h, p, U.UPIR_MAP_FROM)
    want = np.arange(1024, dtype=np.float32)
    want[16:32] = -1
    assert np.array_equal(v, want)


# --------------------------------------------------------- small matmul ----

@pytest.mark.parametrize("kind,tol", [(U.UPIR_BODY_MATMUL_F32, 1e-5), (U.UPIR_BODY_MATMUL_BF16, 3e-3),
                                      (U.UPIR_BODY_MATMUL_SPLIT3, 1e-5)])
@pytest.mark.parametrize("M,N,K", [(17, 33, 65), (1, 1, 1), (64, 48, 40)])
def test_matmul_generic_parity(ctx, kind, tol, M, N, K):
    A = synth.normal(21, 0, M * K).reshape(M, K)
    B = synth.normal(21, 1, K * N).reshape(K, N)
    tA, tB = dev(A), dev(B)
    tC = torch.zeros(M, N, device="cuda")
    ws = torch.zeros(max(1, U.upir_matmul_workspace_bytes(kind, M, N, K)), dtype=torch.uint8, device="cuda")
    args = U.upir_matmul_args(tA.data_ptr(), tB.data_ptr(), tC.data_ptr(), K, K, N, N, ws.data_ptr(), ws.numel())
    lp = ctx.loop(kind, args, [(0, M, 1), (0, N, 1)], H.make_sched(U.UPIR_SCHED_STATIC), None)
    ctx.launch(lp, H.make_spmd(3, 64))
    ctx.sync()
    C_ = tC.cpu().numpy()
    assert bodies.frob_rel(C_, bodies.matmul(A, B)) <= tol
    if kind != U.UPIR_BODY_MATMUL_F32:
        # workspace regions of M x K' (A) and N x K' (B) elements, K' = K
        # rounded up to 32; the generic kernel's layout is rows of K in each
        w = ws.cpu().numpy().view(np.uint16)
        Kp = (K + 31) // 32 * 32
        ah = w[:M * K].reshape(M, K)
        bh = w[M * Kp:M * Kp + N * K].reshape(N, K)
        hiA, loA = bodies.split_bf16(A)
        hiB, loB = bodies.split_bf16(B)
        assert np.array_equal(ah, (hiA.view(np.uint32) >> 16).astype(np.uint16))
        assert np.array_equal(bh, (hiB.T.view(np.uint32) >> 16).astype(np.uint16))
        if kind == U.UPIR_BODY_MATMUL_SPLIT3:
            al = w[(M + N) * Kp:(M + N) * Kp + M * K].reshape(M, K)
            bl = w[(2 * M + N) * Kp:(2 * M + N) * Kp + N * K].reshape(N, K)
            assert np.array_equal(al, (loA.view(np.uint32) >> 16).astype(np.uint16))
            assert np.array_equal(bl, (np.ascontiguousarray(loB.T).view(np.uint32) >> 16).astype(np.uint16))
        emul = bodies.matmul_bf16(A, B) if kind == U.UPIR_BODY_MATMUL_BF16 else bodies.matmul_split3(A, B)
        assert bodies.frob_rel(C_, emul) <= 1e-5
    ctx.free(lp)


def test_matmul_integer_exact(ctx):
    rng = np.random.default_rng(4)
    M, N, K = 40, 24, 72
    A = rng.integers(-2, 3, (M, K)).astype(np.float32)
    B = rng.integers(-2, 3, (K, N)).astype(np.float32)
    want = bodies.matmul(A, B)
    for kind in (U.UPIR_BODY_MATMUL_F32, U.UPIR_BODY_MATMUL_BF16, U.UPIR_BODY_MATMUL_SPLIT3):
        tA, tB = dev(A), dev(B)
        tC = torch.zeros(M, N, device="cuda")
        args = U.upir_matmul_args(tA.data_ptr(), tB.data_ptr(), tC.data_ptr(), K, K, N, N, None, 0)
        lp = ctx.loop(kind, args, [(0, M, 1), (0, N, 1)], H.make_sched(U.UPIR_SCHED_STATIC_CHUNK, 5), None)
        ctx.launch(lp, H.make_spmd(4, 64))
        ctx.sync()
        assert np.array_equal(tC.cpu().numpy().astype(np.float64), want)
        ctx.free(lp)


def test_jacobi_full_size_benchmark_configuration(ctx):
    """The benchmark's workload at full size: 4096 x 4096, zero boundary,
    interior uniform [0, 1), 100 sweeps as one captured graph with async
    (deferred-fold) max residuals, in the tuned launch configuration the
    benchmark times (tile 64 x 256, 256 units). Grid and all 100 residuals
    bit-exact against the oracle."""
    N, sweeps = 4096, 100
    u0 = jacobi_grid(N, N, seed=12345)
    a, b = dev(u0), dev(u0)
    res = torch.zeros(sweeps, dtype=torch.float64, device="cuda")
    sched = H.make_sched(U.UPIR_SCHED_STATIC, tile=(64, 256))
    spmd = H.make_spmd(0, 256)
    hs = []
    for k in range(sweeps):
        src, dst = (a, b) if k % 2 == 0 else (b, a)
        hs.append(ctx.loop(U.UPIR_BODY_JACOBI5, U.upir_jacobi5_args(src.data_ptr(), dst.data_ptr(), N),
                           [(1, N - 1, 1), (1, N - 1, 1)], sched,
                           H.make_red(U.UPIR_RED_MAX, res[k:].data_ptr(), async_=True)))
    assert U.VARIANTS[ctx.resolve(hs[0], spmd)[2]] == "jacobi_tile"
    ctx.launch(hs, spmd)
    ctx.sync()
    a.copy_(dev(u0))
    b.copy_(dev(u0))
    res.zero_()
    torch.cuda.synchronize()
    ctx.graph_begin()
    ctx.launch(hs, spmd)
    g = ctx.graph_end()
    ctx.graph_launch(g)
    ctx.sync()
    want_u, want_r = bodies.jacobi5(u0, sweeps)
    assert np.array_equal(a.cpu().numpy(), want_u)
    assert np.array_equal(res.cpu().numpy(), want_r)
    ctx.graph_destroy(g)
    for h in hs:
        ctx.free(h)


def test_jacobi_beyond_last_level_cache(ctx):
    """Two grids larger than the 256 MB cache (2 x 151 MB): the sweep stores
    with the non-temporal hint. Three sweeps with async max residuals, grid
    and residuals bit-exact against the oracle."""
    Hh, W, sweeps = 8192, 4612, 3
    note(f"jacobi {Hh}x{W} beyond the cache")
    u0 = jacobi_grid(Hh, W, seed=41)
    a, b = dev(u0), dev(u0)
    res = torch.zeros(sweeps, dtype=torch.float64, device="cuda")
    hs = []
    for k in range(sweeps):
        src, dst = (a, b) if k % 2 == 0 else (b, a)
        hs.append(ctx.loop(U.UPIR_BODY_JACOBI5, U.upir_jacobi5_args(src.data_ptr(), dst.data_ptr(), W),
                           [(1, Hh - 1, 1), (1, W - 1, 1)], None,
                           H.make_red(U.UPIR_RED_MAX, res[k:].data_ptr(), async_=True)))
    assert U.VARIANTS[ctx.resolve(hs[0])[2]] == "jacobi_tile"
    assert 2 * Hh * W * 4 > 256 << 20
    ctx.launch(hs)
    ctx.sync()
    want_u, want_r = bodies.jacobi5(u0, sweeps)
    assert np.array_equal(b.cpu().numpy(), want_u)
    assert np.array_equal(res.cpu().numpy(), want_r)
    for h in hs:
        ctx.free(h)
    del a, b
    torch.cuda.empty_cache()


def test_axpy_beyond_int32_indices(ctx):
    """n = 2^31 + 17 (16 GiB of operands): 64-bit iteration indices through
    the non-temporal streaming kernel. Outputs at 2,000 sampled indices and
    around the 2^31 boundary are bit-exact against the oracle computed on
    those elements; the float64 sum is checked against an independent
    float64 reduction of the outputs (torch) within the float sum bound."""
    n = (1 << 31) + 17
    note(f"axpy n={n}")
    x = torch.empty(n, device="cuda")
    y = torch.empty(n, device="cuda")
    c = 1 << 28
    for s0 in range(0, n, c):
        m = min(c, n - s0)
        x[s0:s0 + m] = synth.uniform_pm1_torch(61, 0, m, start=s0, device="cuda")
        y[s0:s0 + m] = synth.uniform_pm1_torch(61, 1, m, start=s0, device="cuda")
    torch.cuda.synchronize()  # the library runs on its own stream
    r = dbl()
    lp = ctx.loop(U.UPIR_BODY_AXPY, U.upir_axpy_args(2.5, 0, x.data_ptr(), y.data_ptr()), [(0, n, 1)], None,
                  H.make_red(U.UPIR_RED_SUM, r.data_ptr()))
    assert U.VARIANTS[ctx.resolve(lp)[2]] == "stream4"
    ctx.launch(lp)
    ctx.sync()
    rng = np.random.default_rng(61)
    idx = np.unique(np.concatenate([rng.integers(0, n, 2000), [0, 1, (1 << 31) - 2, (1 << 31) - 1, 1 << 31,
                                                                   (1 << 31) + 1, n - 2, n - 1]]))
    got = y[torch.from_numpy(idx).cuda()].cpu().numpy()
    xs = np.array([synth.uniform_pm1(61, 0, 1, start=int(i))[0] for i in idx], np.float32)
    ys = np.array([synth.uniform_pm1(61, 1, 1, start=int(i))[0] for i in idx], np.float32)
    assert np.array_equal(got, bodies.axpy(2.5, xs, ys))
    want_s = float(y.double().sum().item())
    abs_s = float(y.double().abs().sum().item())
    assert abs(r.item() - want_s) <= 1e-5 * abs_s
    ctx.free(lp)
    del x, y
    torch.cuda.empty_cache()


def test_stencils_with_empty_interior(ctx):
    """Grids too small for an interior: nothing is written, a reduction
    returns its init."""
    u = np.arange(4, dtype=np.float32).reshape(2, 2)
    a, b = dev(u), dev(np.full((2, 2), -1.0, np.float32))
    r = dbl()
    lp = ctx.loop(U.UPIR_BODY_JACOBI5, U.upir_jacobi5_args(a.data_ptr(), b.data_ptr(), 2), [(1, 1, 1), (1, 1, 1)],
                  None, H.make_red(U.UPIR_RED_MAX, r.data_ptr(), init=0.5))
    ctx.launch(lp)
    ctx.sync()
    assert (b.cpu().numpy() == -1.0).all() and r.item() == 0.5
    ctx.free(lp)
    s6 = dev(np.ones((6, 8), np.float32))
    d6 = dev(np.full((6, 8), -1.0, np.float32))
    w = dev(np.ones(49, np.float32))
    lf = ctx.loop(U.UPIR_BODY_FILTER7, U.upir_filter7_args(s6.data_ptr(), d6.data_ptr(), w.data_ptr(), 8),
                  [(3, 3, 1), (3, 5, 1)])
    ctx.launch(lf)
    ctx.sync()
    assert (d6.cpu().numpy() == -1.0).all()
    ctx.free(lf)
