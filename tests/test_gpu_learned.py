"""GPU checks of schedule selection: the cost-model kernels against the
float64 oracle, the tuner's bookkeeping, and what the trained model gains.

Forward outputs and every parameter gradient must match the oracle's
float64 values normwise within 1e-5 on the same batch; one Adam step must
match the oracle's update within 1e-6 normwise. The tuner must leave the
loop's outputs untouched and AUTO must then resolve to the measured best.
The gain tests train on a timing table of loops and task graphs and check
that on held-out loops the model's choices are faster than the library
default, and that on a task graph it never saw the batched executor with the
model's engine schedule comes within 5% of the exhaustive tuner's best and
beats one launch per task.
"""
import ctypes as C
import os
import sys
import tempfile

import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from paper_2209_10643_amd import helpers as H
from paper_2209_10643_amd import upir as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = {"W1": (64, 32), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (1, 64), "b3": (1,)}


def note(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    U.lib()
    s = torch.cuda.Stream()
    torch.cuda.set_stream(s)
    c = H.Context(0, stream=s)
    yield c
    c.close()


def flat(P):
    return np.concatenate([np.asarray(P[k], np.float32).ravel() for k in omlp.NAMES])


def unflat(v):
    P, o = {}, 0
    for k in omlp.NAMES:
        n = int(np.prod(SHAPES[k]))
        P[k] = np.asarray(v[o:o + n], np.float64).reshape(SHAPES[k])
        o += n
    return P


def params(seed=3):
    P = {}
    for i, k in enumerate(omlp.NAMES):
        n = int(np.prod(SHAPES[k]))
        P[k] = (synth.uniform_pm1(seed, i, n).astype(np.float64) * 0.3).reshape(SHAPES[k])
    return P


def batch(seed, n):
    X = synth.uniform_pm1(seed, 50, n * 32).reshape(n, 32).astype(np.float32)
    t = (synth.uniform_pm1(seed, 51, n) * 4).astype(np.float32)
    return X, t


def nrel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_mlp_forward_matches_oracle(ctx):
    P = params()
    U.upir_model_init(ctx.h, 1)
    v = flat(P)
    U.upir_model_set_params(ctx.h, v.ctypes.data_as(C.POINTER(C.c_float)))
    X, _ = batch(4, 1000)
    tX = torch.from_numpy(X).cuda()
    tY = torch.zeros(1000, device="cuda")
    U.upir_model_forward(ctx.h, tX.data_ptr(), 1000, tY.data_ptr())
    ctx.sync()
    want, _ = omlp.forward(unflat(v), X)
    assert nrel(tY.cpu().numpy(), want) <= 1e-5


@pytest.mark.parametrize("n", [256, 77])
def test_mlp_gradients_match_oracle(ctx, n):
    P = params(5)
    v = flat(P)
    U.upir_model_init(ctx.h, 1)
    U.upir_model_set_params(ctx.h, v.ctypes.data_as(C.POINTER(C.c_float)))
    X, t = batch(6, n)
    tX, tt = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    g = torch.zeros(U.UPIR_MLP_PARAMS, device="cuda")
    loss = C.c_float()
    U.upir_model_step(ctx.h, tX.data_ptr(), tt.data_ptr(), n, 1e-3, 0, g.data_ptr(), C.byref(loss))
    got = unflat(g.cpu().numpy())
    Pd = unflat(v)
    want = omlp.backward(Pd, X, t)
    for k in omlp.NAMES:
        assert nrel(got[k], want[k]) <= 1e-5, k
    assert abs(loss.value - omlp.loss(Pd, X, t)) <= 1e-5 * omlp.loss(Pd, X, t)
    # no Adam step was taken: parameters unchanged
    back = np.zeros(U.UPIR_MLP_PARAMS, np.float32)
    U.upir_model_get_params(ctx.h, back.ctypes.data_as(C.POINTER(C.c_float)))
    assert np.array_equal(back, v)


def test_adam_steps_match_oracle(ctx):
    P = params(7)
    v = flat(P)
    U.upir_model_init(ctx.h, 1)
    U.upir_model_set_params(ctx.h, v.ctypes.data_as(C.POINTER(C.c_float)))
    Pd, m, vv = unflat(v), omlp.zeros_like(unflat(v)), omlp.zeros_like(unflat(v))
    for step in range(1, 4):
        X, t = batch(10 + step, 128)
        tX, tt = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
        U.upir_model_step(ctx.h, tX.data_ptr(), tt.data_ptr(), 128, 1e-3, 1, None, None)
        g = omlp.backward(Pd, X, t)
        Pd, m, vv = omlp.adam_step(Pd, g, m, vv, step, lr=1e-3)
    got = np.zeros(U.UPIR_MLP_PARAMS, np.float32)
    U.upir_model_get_params(ctx.h, got.ctypes.data_as(C.POINTER(C.c_float)))
    # compare the parameter change (float32 parameters, float64 oracle)
    assert nrel(got.astype(np.float64) - v, flat(Pd).astype(np.float64) - v) <= 1e-4
    assert nrel(got, flat(Pd)) <= 1e-6


def test_model_and_table_files_round_trip(ctx):
    U.upir_model_init(ctx.h, 99)
    a = np.zeros(U.UPIR_MLP_PARAMS, np.float32)
    U.upir_model_get_params(ctx.h, a.ctypes.data_as(C.POINTER(C.c_float)))
    # Kaiming-uniform bounds
    assert np.abs(a[:2048]).max() <= np.sqrt(6 / 32) and np.abs(a[2048 + 64:2048 + 64 + 4096]).max() <= np.sqrt(6 / 64)
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "m.bin").encode()
        U.upir_model_save(ctx.h, p)
        U.upir_model_init(ctx.h, 1)
        U.upir_model_load(ctx.h, p)
        b = np.zeros_like(a)
        U.upir_model_get_params(ctx.h, b.ctypes.data_as(C.POINTER(C.c_float)))
        assert np.array_equal(a, b)


def test_tuner_keeps_outputs_and_auto_takes_best(ctx):
    n = 300007
    x = torch.from_numpy(synth.uniform_pm1(8, 0, n)).cuda()
    y0 = synth.uniform_pm1(8, 1, n)
    y = torch.from_numpy(y0.copy()).cuda()
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    lp = ctx.loop(U.UPIR_BODY_AXPY, U.upir_axpy_args(2.5, 0, x.data_ptr(), y.data_ptr()), [(0, n, 1)], None,
                  H.make_red(U.UPIR_RED_SUM, r.data_ptr()))
    n0 = C.c_int64()
    U.upir_tune_db_size(ctx.h, C.byref(n0))
    cnt = C.c_int32()
    U.upir_candidates(ctx.h, lp, C.byref(cnt))
    best_s, best_p, us = U.upir_sched(), U.upir_spmd(), C.c_double()
    U.upir_tune(ctx.h, None, lp, 3, C.byref(best_s), C.byref(best_p), C.byref(us))
    n1 = C.c_int64()
    U.upir_tune_db_size(ctx.h, C.byref(n1))
    assert n1.value - n0.value == cnt.value >= 2
    ctx.sync()
    assert np.array_equal(y.cpu().numpy(), y0)          # timing ran on a copy
    sp, sc, _ = ctx.resolve(lp)
    assert (sp.num_teams, sp.num_units, sc.policy, sc.chunk) == \
        (best_p.num_teams, best_p.num_units, best_s.policy, best_s.chunk)
    assert us.value > 0
    ctx.free(lp)


@pytest.fixture(scope="module")
def trained(ctx):
    """Tune the loop population and the training task graphs, train the cost
    model on the GPU (20% of loops and graphs held out), leave it enabled."""
    import bench
    res = bench.learned_schedule(torch, ctx, n_random=120, reps=3, epochs=120, log_every=0)
    note(res)
    return res


def test_training_gains_over_default(ctx, trained):
    """On held-out loops the model's choices are faster than the library
    default: overall, and on the loops where the default is measurably not
    the best candidate (where a choice can gain)."""
    res = trained
    assert res["mse_final_train_holdout"][0] < res["mse_initial_train_holdout"][0]
    assert res["mse_final_train_holdout"][1] < res["mse_initial_train_holdout"][1]
    assert res["holdout_gain_vs_default_geomean"] > 1.0
    assert res["holdout_loops_default_not_best"] >= 10
    assert res["holdout_gain_where_default_not_best_geomean"] > 1.0


def test_batched_learned_beats_plain_near_tuner(ctx, trained):
    """The benchmark's 2048-task graph, never tuned nor trained on: the
    batched executor with the model's engine schedule is within 5% of the
    exhaustive batch tuner's best schedule (the slowest candidates cost 10 to
    30% more) and far faster than one launch per task, at equal accuracy.
    (Against the default schedule the model gains 0 to 4% on this graph from
    run to run: the default is itself within a few percent of the best.)"""
    import bench
    res = bench.bench_batched(torch, ctx, bench.Timer(torch, torch.cuda.current_stream()), have_model=True)
    note({k: v for k, v in res.items() if k != "vs_oracle"})
    assert res["learned_source"] == "cost model"
    assert res["batched_equals_plain_at_tol"]
    assert res["vs_oracle"]["axpy_bitexact"]
    assert res["vs_oracle"]["sum_max_err_over_l1"] <= 1e-5 and res["vs_oracle"]["matvec_max_normwise_err"] <= 1e-5
    assert res["learned_regret_vs_tuner"] <= 1.05
    assert res["learned_vs_plain_speedup"] > 5.0
