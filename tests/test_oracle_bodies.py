"""Pins of the oracle's loop bodies and reductions (CPU only).

Each pin rests on something other than the oracle itself: exact rational
arithmetic, integer closed forms, fixed points and eigenmodes of the Jacobi
iteration, integer matrices, and per-point brute force in Python scalars.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import synth
from oracle import bodies, reduce


def _rn32_exact(v: F) -> np.float32:
    """Round a rational to float32, nearest-even, by comparing neighbours."""
    f = np.float32(float(v))
    cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]

    def key(t):
        odd = int(np.array([t], np.float32).view(np.uint32)[0]) & 1
        return (abs(F(float(t)) - v), odd)
    return min(cands, key=key)


# ---------------------------------------------------------------- AXPY ----

def test_fma_f32_matches_exact_rationals():
    rng = np.random.default_rng(1)
    a = rng.standard_normal(3000).astype(np.float32)
    x = (rng.standard_normal(3000) * 2.0 ** rng.integers(-30, 30, 3000)).astype(np.float32)
    y = (rng.standard_normal(3000) * 2.0 ** rng.integers(-30, 30, 3000)).astype(np.float32)
    for i in range(3000):
        got = bodies.fma_f32(a[i], x[i:i + 1], y[i:i + 1])[0]
        want = _rn32_exact(F(float(a[i])) * F(float(x[i])) + F(float(y[i])))
        assert got == want, i


def test_fma_f32_double_rounding_case():
    # a*x = 2^-24 - 2^-70, y = 1 + 2^-23: float64 rounds the sum onto the
    # float32 midpoint 1 + 2^-23 + 2^-24 and ties-to-even would go up; the
    # exact value is below the midpoint, so the answer is 1 + 2^-23.
    a = np.float32(1 + 2.0 ** -23)
    x = np.float32(2.0 ** -24 * (1 - 2.0 ** -23))
    y = np.float32(1 + 2.0 ** -23)
    naive = np.float32(np.float64(a) * np.float64(x) + np.float64(y))
    got = bodies.fma_f32(a, np.array([x]), np.array([y]))[0]
    assert got == np.float32(1 + 2.0 ** -23)
    assert naive != got


def test_axpy_on_input_grid_is_exact():
    # inputs on the 2^-23 grid, a = 2.5: a*x + y is a multiple of 2^-24 below 4,
    # so it fits in 26 bits; the float32 result equals the exact value rounded once.
    n = 4096
    x = synth.uniform_pm1(12345, 0, n)
    y = synth.uniform_pm1(12345, 1, n)
    got = bodies.axpy(2.5, x, y)
    for i in range(0, n, 97):
        assert got[i] == _rn32_exact(F(5, 2) * F(float(x[i])) + F(float(y[i])))


def test_sum_closed_forms():
    for n in (0, 1, 63, 64, 65, 1000, 2 ** 20 + 3):
        v = np.arange(n, dtype=np.float32)  # exact integers below 2^24
        if n <= 2 ** 24:
            assert bodies.sum_f64(v) == n * (n - 1) // 2
    assert reduce.reduce(reduce.SUM, np.arange(10 ** 6, dtype=np.int64)) == 10 ** 6 * (10 ** 6 - 1) // 2


def test_sum_is_exact_rational_sum():
    rng = np.random.default_rng(2)
    v = (rng.standard_normal(500) * 2.0 ** rng.integers(-40, 40, 500)).astype(np.float32)
    exact = sum((F(float(t)) for t in v), F(0))
    assert bodies.sum_f64(v) == float(exact)


def test_reduce_ops():
    v = np.array([3.0, -7.5, 2.25], np.float32)
    assert reduce.reduce(reduce.MAX, v) == 3.0
    assert reduce.reduce(reduce.MIN, v) == -7.5
    assert reduce.reduce(reduce.MAX, v, init=10.0) == 10.0
    assert reduce.reduce(reduce.SUM, v, init=1.0) == -1.25
    assert reduce.reduce(reduce.MAX, np.array([], np.float32)) is None


# -------------------------------------------------------------- Jacobi ----

def _jacobi_brute(u):
    """One float32 sweep point by point with numpy float32 scalars."""
    H, W = u.shape
    out = u.copy()
    q = np.float32(0.25)
    for i in range(1, H - 1):
        for j in range(1, W - 1):
            out[i, j] = ((u[i - 1, j] + u[i + 1, j]) + (u[i, j - 1] + u[i, j + 1])) * q
    return out


@pytest.mark.parametrize("H,W", [(5, 7), (33, 65), (3, 3), (2, 9)])
def test_jacobi_brute_force(H, W):
    u = synth.uniform_01(3, 0, H * W).reshape(H, W)
    u[0, :] = u[-1, :] = 0
    u[:, 0] = u[:, -1] = 0
    got, res = bodies.jacobi5(u, 3)
    ref = u.copy()
    rr = []
    for _ in range(3):
        nxt = _jacobi_brute(ref)
        m = 0.0
        for i in range(1, H - 1):
            for j in range(1, W - 1):
                m = max(m, abs(float(nxt[i, j]) - float(ref[i, j])))
        rr.append(m)
        ref = nxt
    assert np.array_equal(got, ref)
    assert res.tolist() == rr


@pytest.mark.parametrize("H,W", [(5, 7), (9, 4)])
def test_jacobi_min_and_sum_residual_brute_force(H, W):
    """min and sum of |u1 - u0| point by point; the sum is compared with the
    exact rational sum rounded once (what a correctly rounded sum returns)."""
    from fractions import Fraction
    u = synth.uniform_01(5, 1, H * W).reshape(H, W)
    u[0, :] = u[-1, :] = 0
    u[:, 0] = u[:, -1] = 0
    _, rmin = bodies.jacobi5(u, 2, op="min")
    _, rsum = bodies.jacobi5(u, 2, op="sum")
    ref = u.copy()
    for k in range(2):
        nxt = _jacobi_brute(ref)
        ds = [abs(Fraction(float(nxt[i, j])) - Fraction(float(ref[i, j])))
              for i in range(1, H - 1) for j in range(1, W - 1)]
        assert rmin[k] == float(min(ds))
        assert rsum[k] == float(sum(ds))
        ref = nxt


def test_jacobi_residual_ops_on_impulse_and_empty():
    u = np.zeros((7, 7), np.float32)
    u[3, 3] = 1
    # one sweep: the impulse point drops by 1, its four neighbours rise by 1/4
    assert bodies.jacobi5(u, 1, op="sum")[1][0] == 2.0
    assert bodies.jacobi5(u, 1, op="min")[1][0] == 0.0
    e = np.zeros((2, 5), np.float32)
    assert bodies.update_f64(e, e, "min") == math.inf
    assert bodies.update_f64(e, e, "sum") == 0.0 == bodies.update_f64(e, e, "max")


def test_jacobi_linear_field_fixed_point():
    N = 64
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    u = (i + 2 * j).astype(np.float32)
    got, res = bodies.jacobi5(u, 5)
    assert np.array_equal(got, u) and (res == 0).all()


def test_jacobi_zero_and_impulse():
    z = np.zeros((9, 9), np.float32)
    g, r = bodies.jacobi5(z, 2)
    assert not g.any() and (r == 0).all()
    u = np.zeros((9, 9), np.float32)
    u[4, 4] = 1
    g, r = bodies.jacobi5(u, 1)
    assert g[4, 4] == 0 and g[3, 4] == g[5, 4] == g[4, 3] == g[4, 5] == 0.25
    assert g.sum() == 1.0 and r[0] == 1.0


def test_jacobi_eigenmode_decay_f64():
    N, p, q, k = 65, 2, 3, 7
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    h = math.pi / (N - 1)
    u = np.sin(p * h * i) * np.sin(q * h * j)
    lam = (math.cos(p * h) + math.cos(q * h)) / 2
    got, _ = bodies.jacobi5(u, k, mode="f64")
    assert np.abs(got - lam ** k * u).max() < 1e-12


# ------------------------------------------------------------- filter7 ----

def test_filter7_brute_force_exact_rationals():
    """Every interior point: 49 fused multiply-adds in filter order, each the
    exact rational a*x + s rounded once to float32."""
    H, W = 9, 11
    src = synth.uniform_pm1(30, 0, H * W).reshape(H, W)
    w = synth.uniform_pm1(30, 1, 49).reshape(7, 7)
    dst0 = synth.uniform_pm1(30, 2, H * W).reshape(H, W)
    got = bodies.filter7(src, w, dst0)
    for i in range(H):
        for j in range(W):
            if 3 <= i < H - 3 and 3 <= j < W - 3:
                acc = np.float32(0)
                for m in range(7):
                    for n in range(7):
                        acc = _rn32_exact(F(float(w[m, n])) * F(float(src[i + m - 3, j + n - 3])) + F(float(acc)))
                assert got[i, j] == acc, (i, j)
            else:
                assert got[i, j] == dst0[i, j], (i, j)


def test_filter7_delta_shift_and_constant():
    H, W = 20, 23
    src = synth.uniform_pm1(31, 0, H * W).reshape(H, W)
    delta = np.zeros((7, 7), np.float32)
    delta[3, 3] = 1
    assert np.array_equal(bodies.filter7(src, delta), src)          # identity
    shift = np.zeros((7, 7), np.float32)
    shift[1, 5] = 1                                                   # row -2, column +2
    got = bodies.filter7(src, shift)
    assert np.array_equal(got[3:-3, 3:-3], src[1:-5, 5:-1])
    # constant field, weights on the 2^-6 grid: every partial sum is exact
    w = np.round(synth.uniform_pm1(31, 1, 49) * 64).astype(np.float32).reshape(7, 7) / 64
    c = np.float32(0.75)
    got = bodies.filter7(np.full((H, W), c, np.float32), w)
    total = sum(F(float(v)) for v in w.ravel()) * F(float(c))
    assert (got[3:-3, 3:-3] == np.float32(float(total))).all()


def test_filter7_small_arrays_unchanged():
    for H, W in [(6, 9), (9, 6), (1, 1)]:
        a = synth.uniform_pm1(32, 0, H * W).reshape(H, W)
        assert np.array_equal(bodies.filter7(a, np.ones((7, 7), np.float32)), a)


# -------------------------------------------------------------- matmul ----

def test_matmul_integer_brute_force():
    rng = np.random.default_rng(4)
    for (M, K, N) in [(1, 1, 1), (17, 33, 65), (5, 128, 3)]:
        A = rng.integers(-2, 3, (M, K)).astype(np.float32)
        B = rng.integers(-2, 3, (K, N)).astype(np.float32)
        C = bodies.matmul(A, B)
        Ai, Bi = A.astype(int).tolist(), B.astype(int).tolist()
        for i in range(M):
            for j in range(N):
                assert C[i, j] == sum(Ai[i][k] * Bi[k][j] for k in range(K))
        # integer entries are bfloat16-exact: every variant is exact
        assert np.array_equal(bodies.matmul_bf16(A, B), C)
        assert np.array_equal(bodies.matmul_split3(A, B), C)


def test_matmul_identity_and_entry():
    A = synth.normal(5, 0, 24 * 24).reshape(24, 24)
    I = np.eye(24, dtype=np.float32)
    assert np.array_equal(bodies.matmul(A, I), A.astype(np.float64))
    B = synth.normal(5, 1, 24 * 24).reshape(24, 24)
    C = bodies.matmul(A, B)
    for (i, j) in [(0, 0), (3, 17), (23, 23)]:
        exact = sum((F(float(A[i, k])) * F(float(B[k, j])) for k in range(24)), F(0))
        assert abs(bodies.matmul_entry(A, B, i, j) - float(exact)) <= abs(float(exact)) * 2.0 ** -52
        assert abs(C[i, j] - float(exact)) <= 1e-12 * max(1.0, abs(float(exact)))


def _bf16_round_fraction(x) -> F:
    """Nearest bfloat16 (8 significant bits, ties to even) of a finite,
    normal-range value, computed on exact rationals: scale by the bfloat16
    ulp of x's binade and round the quotient to the nearest integer."""
    fx = F(float(x))
    if fx == 0:
        return F(0)
    e = math.floor(math.log2(abs(float(fx))))
    ulp = F(2) ** (e - 7)
    q = fx / ulp
    fl = q.numerator // q.denominator
    rem = q - fl
    if rem > F(1, 2) or (rem == F(1, 2) and fl % 2 == 1):
        fl += 1
    return fl * ulp


def test_matmul_bf16_and_split3_closed_form_one_by_one():
    # a = 1 + 2^-9: its bfloat16 rounding is 1 (2^-9 is below half an ulp of
    # 1, which is 2^-7) and the residual 2^-9 is a bfloat16 number, so the
    # one-pass product of the roundings is exactly 1 and the three-pass split
    # product lo*hi + hi*lo + hi*hi is exactly 1 + 2^-8 (the true product is
    # 1 + 2^-8 + 2^-18: the split drops only lo*lo).
    a = np.array([[1 + 2 ** -9]], np.float32)
    assert bodies.matmul_bf16(a, a)[0, 0] == 1.0
    assert bodies.matmul_split3(a, a)[0, 0] == 1 + 2 ** -8
    assert bodies.matmul(a, a)[0, 0] == (1 + 2 ** -9) ** 2


def test_matmul_bf16_and_split3_exact_rationals():
    # non-integer 2 x 3 and 3 x 2 operands whose entries all have distinct
    # high and low bfloat16 parts; both compositions checked entry by entry
    # against exact rational arithmetic on an independent rounding
    A = np.array([[1.2345678, -0.3141593, 7.0001],
                  [2.5e-3, -19.75003, 0.6666667]], np.float32)
    B = np.array([[0.1, -2.7182817],
                  [1.4142135, 33.333336],
                  [-0.0078125001, 5.55555]], np.float32)
    hiA = [[_bf16_round_fraction(v) for v in r] for r in A]
    hiB = [[_bf16_round_fraction(v) for v in r] for r in B]
    loA = [[_bf16_round_fraction(float(F(float(v)) - h)) for v, h in zip(r, hr)] for r, hr in zip(A, hiA)]
    loB = [[_bf16_round_fraction(float(F(float(v)) - h)) for v, h in zip(r, hr)] for r, hr in zip(B, hiB)]
    for r in range(2):
        for c in range(3):
            assert loA[r][c] != 0 and hiA[r][c] != F(float(A[r, c]))
    Cb = bodies.matmul_bf16(A, B)
    Cs = bodies.matmul_split3(A, B)
    for i in range(2):
        for j in range(2):
            one = sum((hiA[i][k] * hiB[k][j] for k in range(3)), F(0))
            three = sum((loA[i][k] * hiB[k][j] + hiA[i][k] * loB[k][j] + hiA[i][k] * hiB[k][j]
                         for k in range(3)), F(0))
            # three float64 products of bfloat16 values are exact; the sums
            # round at most once per addition
            assert abs(F(float(Cb[i, j])) - one) <= abs(one) * F(2) ** -50
            assert abs(F(float(Cs[i, j])) - three) <= abs(three) * F(2) ** -49
            # and they differ from each other and from the unrounded product
            exact = sum((F(float(A[i, k])) * F(float(B[k, j])) for k in range(3)), F(0))
            assert Cb[i, j] != Cs[i, j]
            assert abs(three - exact) < abs(one - exact)


def _bf16_exact(x: np.float32) -> np.float32:
    """Nearest bfloat16 by brute force over the two truncation neighbours."""
    b = int(np.array([x], np.float32).view(np.uint32)[0])
    lo = b & 0xFFFF0000
    hi = (lo + 0x10000) & 0xFFFFFFFF
    vlo = np.array([lo], np.uint32).view(np.float32)[0]
    vhi = np.array([hi], np.uint32).view(np.float32)[0]
    if not np.isfinite(x):
        return x
    fx = F(float(x))
    dlo = abs(F(float(vlo)) - fx)
    dhi = abs(F(float(vhi)) - fx) if np.isfinite(vhi) else None
    if dhi is None:
        # rounding past the largest finite bf16 goes to infinity when at/above the midpoint
        top = abs(F(float(vlo))) + F(2) ** (int(math.floor(math.log2(abs(float(vlo))))) - 7) / 2
        return vlo if abs(fx) < top else np.float32(math.copysign(math.inf, float(x)))
    if dlo < dhi:
        return vlo
    if dhi < dlo:
        return vhi
    return vlo if ((lo >> 16) & 1) == 0 else vhi


def test_rne_bf16_brute_force():
    rng = np.random.default_rng(6)
    bits = rng.integers(0, 2 ** 32, 20000, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    # add ties, tiny, subnormal, signed zero and near-overflow values
    extra = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, -0.0, 1e-40, -3e-39,
                      3.3895313892515355e38, 3.4028234663852886e38, -3.39e38], np.float32)
    x = np.concatenate([x, extra])
    got = bodies.rne_bf16(x)
    for i in range(len(x)):
        want = _bf16_exact(x[i])
        assert got[i] == want or (got[i] == 0 and want == 0), (x[i], got[i], want)
        assert np.signbit(got[i]) == np.signbit(want)
    assert np.isnan(bodies.rne_bf16(np.array([np.nan], np.float32))[0])
    assert bodies.rne_bf16(np.array([np.inf], np.float32))[0] == np.inf


def test_split_bf16_reconstructs():
    x = synth.normal(7, 0, 100000)
    hi, lo = bodies.split_bf16(x)
    assert (np.array(hi).view(np.uint32) & 0xFFFF == 0).all()
    assert (np.array(lo).view(np.uint32) & 0xFFFF == 0).all()
    rel = np.abs((hi.astype(np.float64) + lo) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -16
    # the residual x - hi is exact in float32
    r32 = (x - hi).astype(np.float64)
    assert np.array_equal(r32, x.astype(np.float64) - hi.astype(np.float64))


def test_matvec_brute_force():
    A = synth.uniform_pm1(8, 0, 7 * 256).reshape(7, 256)
    x = synth.uniform_pm1(8, 1, 256)
    y = bodies.matvec(A, x)
    for r in range(7):
        exact = sum((F(float(A[r, c])) * F(float(x[c])) for c in range(256)), F(0))
        assert bodies.matvec_row(A[r], x) == float(exact)
        # on the 2^-23 grid every product is a multiple of 2^-46 below 1, so
        # the float64 dot product of 256 terms is exact
        assert y[r] == float(exact)


def test_frob_rel():
    C = np.ones((3, 3))
    assert bodies.frob_rel(C, C) == 0
    assert abs(bodies.frob_rel(C * (1 + 1e-3), C) - 1e-3) < 1e-12
