"""Pins of the oracle's task graph, token chain and MLP (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import mlp, tasks


def _golden(golden_dir):
    with open(f"{golden_dir}/splitmix64_seed0.txt") as f:
        return [int(line, 16) for line in f if line.strip() and not line.startswith("#")]


def test_synth_matches_published_splitmix64(golden_dir):
    want = _golden(golden_dir)
    got = [int(v) for v in synth.hash_u64(0, 0, len(want))]
    assert got == want


def test_synth_numpy_torch_agree():
    for seed, stream, n, start in [(12345, 0, 5000, 0), (1, 7, 333, 99), (2, 3, 10, 2 ** 33)]:
        a = synth.uniform_pm1(seed, stream, n, start)
        b = synth.uniform_pm1_torch(seed, stream, n, start).numpy()
        assert np.array_equal(a, b)
        a = synth.uniform_01(seed, stream, n, start)
        b = synth.uniform_01_torch(seed, stream, n, start).numpy()
        assert np.array_equal(a, b)


def test_synth_grids():
    u = synth.uniform_pm1(9, 0, 100000)
    assert u.min() >= -1 and u.max() < 1
    assert np.array_equal(u * 2.0 ** 23, np.round(u * 2.0 ** 23))
    v = synth.uniform_01(9, 1, 100000)
    assert v.min() >= 0 and v.max() < 1
    assert np.array_equal(v.astype(np.float64) * 2.0 ** 24, np.round(v.astype(np.float64) * 2.0 ** 24))
    z = synth.normal(9, 2, 200000).astype(np.float64)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01


def test_tokens_without_predecessors_are_splitmix_outputs(golden_dir):
    # with no predecessors tok[j] = mix64((j+1) G): the (j+1)-th output of
    # SplitMix64 started at state 0
    want = _golden(golden_dir)
    assert tasks.tokens([[] for _ in want]) == want


def test_tokens_chain_by_hand(golden_dir):
    g = _golden(golden_dir)
    preds = [[], [0], [0, 1]]
    tok = tasks.tokens(preds)
    t1 = synth.mix64(g[1] ^ g[0])
    t2 = synth.mix64(synth.mix64(g[2] ^ g[0]) ^ t1)
    assert tok == [g[0], t1, t2]
    # a different predecessor set changes the token
    assert tasks.tokens([[], [], [0, 1]])[2] != t2


def test_depend_rules():
    I, O, IO = tasks.IN, tasks.OUT, tasks.INOUT
    # RAW, WAR, WAW and read-read on one address
    deps = [[("x", O)], [("x", I)], [("x", I)], [("x", IO)], [("x", O)], [("x", I)]]
    assert tasks.depend_edges(deps) == [[], [0], [0], [0, 1, 2], [0, 1, 2, 3], [0, 3, 4]]
    # independent addresses give no edges; several addresses merge
    deps = [[("a", O)], [("b", O)], [("a", I), ("b", I)], [("c", IO)]]
    assert tasks.depend_edges(deps) == [[], [], [0, 1], []]


def test_depend_random_graph_encoding():
    # the batched workload's encoding: out on tok[j], in on tok[i] per chosen edge
    n = 40
    rng = np.random.default_rng(3)
    edges = {j: sorted(int(i) for i in range(j) if rng.random() < 4 / (n - 1)) for j in range(n)}
    deps = [[(("tok", j), tasks.OUT)] + [(("tok", i), tasks.IN) for i in edges[j]] for j in range(n)]
    assert tasks.depend_edges(deps) == [edges[j] for j in range(n)]


def _params(seed=11):
    P = {}
    shapes = {"W1": (64, 32), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (1, 64), "b3": (1,)}
    for s, (k, shp) in enumerate(shapes.items()):
        P[k] = synth.uniform_pm1(seed, s, int(np.prod(shp))).astype(np.float64).reshape(shp) * 0.3
    return P


def test_mlp_backward_finite_differences():
    P = _params()
    X = synth.uniform_pm1(12, 0, 16 * 32).astype(np.float64).reshape(16, 32)
    t = synth.uniform_pm1(12, 1, 16).astype(np.float64)
    g = mlp.backward(P, X, t)
    h = 1e-6
    rng = np.random.default_rng(0)
    for k in mlp.NAMES:
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            Pp = {q: v.copy() for q, v in P.items()}
            Pm = {q: v.copy() for q, v in P.items()}
            Pp[k].reshape(-1)[idx] += h
            Pm[k].reshape(-1)[idx] -= h
            fd = (mlp.loss(Pp, X, t) - mlp.loss(Pm, X, t)) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)), (k, idx, fd, an)


def test_mlp_zero_net_closed_form():
    P = {k: np.zeros_like(v) for k, v in _params().items()}
    P["b3"][:] = 0.5
    X = np.ones((4, 32))
    t = np.array([0.0, 1.0, 2.0, 3.0])
    y, _ = mlp.forward(P, X)
    assert (y == 0.5).all()
    assert mlp.loss(P, X, t) == np.mean((0.5 - t) ** 2)
    g = mlp.backward(P, X, t)
    assert g["b3"][0] == pytest.approx(np.mean(2 * (0.5 - t)))
    for k in ("W1", "b1", "W2", "b2", "W3"):
        assert not g[k].any()


def test_adam_first_step_is_signed_lr():
    P = _params()
    g = {k: synth.uniform_pm1(13, i, v.size).astype(np.float64).reshape(v.shape) + 0.01
         for i, (k, v) in enumerate(P.items())}
    P2, m, v = mlp.adam_step(P, g, mlp.zeros_like(P), mlp.zeros_like(P), 1, lr=1e-3)
    for k in mlp.NAMES:
        # with bias correction the first step is lr * g / (|g| + eps)
        step = P[k] - P2[k]
        assert np.allclose(step, 1e-3 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12, atol=0)
        assert np.allclose(m[k], 0.1 * g[k]) and np.allclose(v[k], 0.001 * g[k] ** 2)


def test_adam_bias_correction_over_five_steps():
    # a constant gradient g gives m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2,
    # so with bias correction every step t = 1..5 moves each parameter by
    # exactly lr * g / (|g| + eps) up to rounding
    P = _params()
    g = {k: synth.uniform_pm1(14, i, v.size).astype(np.float64).reshape(v.shape) + 0.01
         for i, (k, v) in enumerate(P.items())}
    m, v = mlp.zeros_like(P), mlp.zeros_like(P)
    cur = P
    for t in range(1, 6):
        nxt, m, v = mlp.adam_step(cur, g, m, v, t, lr=1e-3)
        for k in mlp.NAMES:
            assert np.allclose(cur[k] - nxt[k], 1e-3 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-9, atol=1e-15), (t, k)
            assert np.allclose(m[k], (1 - 0.9 ** t) * g[k], rtol=1e-12)
            assert np.allclose(v[k], (1 - 0.999 ** t) * g[k] ** 2, rtol=1e-12)
        cur = nxt
    for k in mlp.NAMES:
        assert np.allclose(P[k] - cur[k], 5e-3 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-9, atol=1e-14)


# ------------------------------------------------------------- taskloop ----

@pytest.mark.parametrize("n,g,k", [(100, 7, 0), (100, 0, 7), (100, 30, 5), (100, 0, 500), (5, 10, 0),
                                   (1, 0, 3), (0, 3, 3), (1000003, 4096, 0)])
def test_taskloop_blocks_cover_and_sizes(n, g, k):
    blocks = tasks.taskloop_blocks(n, g, k, default=4)
    if n == 0:
        assert blocks == []
        return
    # contiguous, in order, covering [0, n) exactly once
    assert blocks[0][0] == 0 and blocks[-1][1] == n
    assert all(a[1] == b[0] for a, b in zip(blocks, blocks[1:]))
    sizes = [hi - lo for lo, hi in blocks]
    assert max(sizes) - min(sizes) <= 1 and min(sizes) >= 1
    G = len(blocks)
    if k and not g:
        assert G == min(k, n)
    if g and not k:
        assert G == max(1, n // g)
        if n >= g:                      # OpenMP: at least g and fewer than 2g per task
            assert min(sizes) >= g and max(sizes) < 2 * g
    if g and k:
        assert G == min(k, n, max(1, n // g))


def test_taskloop_siblings_do_not_wait_for_each_other():
    X, Y = 0x100, 0x200
    deps = [[(X, tasks.OUT)],                                   # 0: a task writing X
            [(X, tasks.IN), (Y, tasks.OUT)], [(X, tasks.IN), (Y, tasks.OUT)], [(X, tasks.IN), (Y, tasks.OUT)],
            [(Y, tasks.IN)]]                                    # 4: reads what the taskloop wrote
    groups = [None, 7, 7, 7, None]
    preds = tasks.depend_edges(deps, groups)
    assert preds == [[], [0], [0], [0], [1, 2, 3]]
    # without the grouping the three out-tasks would chain
    assert tasks.depend_edges(deps) == [[], [0], [0, 1], [0, 1, 2], [1, 2, 3]]
    # a one-task taskloop is an ordinary task
    assert tasks.depend_edges(deps[:2], [None, 3]) == tasks.depend_edges(deps[:2])
