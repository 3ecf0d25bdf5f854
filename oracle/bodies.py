"""Loop bodies executed as serial elisions on the CPU.

Paper: sec. 6 prints one loop body, AXPY, three times (OpenMP, OpenACC and
CUDA forms): ``for (i = 0; i < n; i++) y[i] = y[i] + a * x[i]``, the CUDA form
guarding one element per thread with ``if (i < n)``. Sec. 6.2 names three more
offloaded kernels whose source it does not print: matrix multiplication,
matrix-vector multiplication and a 2D stencil. Their plain mathematical
definitions are written out here.

Readings (the paper is silent or inconsistent):

* AXPY: the scalar is float (the paper's ``int a`` clashes with its float
  arrays and its float64 memrefs); ``y + a*x`` is evaluated as one fused
  multiply-add, i.e. the exact value rounded once to float32.
* Reductions over float32 data are returned in float64.
* Stencil: Jacobi 5-point update ``((N + S) + (W + E)) * 0.25`` on the
  interior, boundary fixed, with the sweep's update max-norm as residual.
* Matmul: row-major C = A B in float64. Every product of two float32
  values is exact in float64; the float64 sums come from a library matrix
  product (its own summation order, rounding error far below every
  tolerance used); ``matmul_entry`` gives one entry correctly rounded.
* BF16 splitting (an extension beyond the paper): ``hi = rne_bf16(a)``,
  ``lo = rne_bf16(a - hi)``.
"""
from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# AXPY and sum (sec. 6, the AXPY listings)
# --------------------------------------------------------------------------

def fma_f32(a, x, y):
    """float32 ``fma(a, x, y)``: the exact value ``a*x + y`` rounded once.

    ``a*x`` of two float32 values is exact in float64 (48 significant bits).
    The float64 sum ``s`` may round; TwoSum gives its exact error ``e``, so
    ``s + e`` is the exact value. Every float32 midpoint is a float64 number,
    so ``s`` and the exact value lie on the same side of every midpoint unless
    ``s`` is itself a midpoint. Hence rounding ``s`` to float32 is right,
    except when ``s`` is a midpoint and ``e`` is non-zero: then the exact value
    is past the midpoint on ``e``'s side and takes that neighbour.
    """
    a64 = np.float64(np.float32(a))
    x64 = np.asarray(x, dtype=np.float32).astype(np.float64)
    y64 = np.asarray(y, dtype=np.float32).astype(np.float64)
    p = a64 * x64
    s = p + y64
    bp = s - y64
    e = (p - bp) + (y64 - (s - bp))
    r = s.astype(np.float32)
    r64 = r.astype(np.float64)
    up = np.nextafter(r, np.float32(np.inf))
    dn = np.nextafter(r, np.float32(-np.inf))
    mid_above = (s > r64) & (s - r64 == (up.astype(np.float64) - r64) / 2)
    mid_below = (s < r64) & (r64 - s == (r64 - dn.astype(np.float64)) / 2)
    r = np.where(mid_above & (e > 0), up, r)
    r = np.where(mid_below & (e < 0), dn, r)
    return np.asarray(r, dtype=np.float32)


def axpy(a, x, y):
    """``y'[i] = fma(a, x[i], y[i])`` for i in index order (sec. 6, AXPY)."""
    return fma_f32(a, x, y)


def sum_f64(v) -> float:
    """Correctly rounded float64 value of the exact sum of ``v`` (sec. 5 reduction, '+')."""
    return math.fsum(np.asarray(v, dtype=np.float64).tolist())


def sum_abs_f64(v) -> float:
    return math.fsum(np.abs(np.asarray(v, dtype=np.float64)).tolist())


# --------------------------------------------------------------------------
# Jacobi 5-point stencil (sec. 6.2 names a 2D stencil; definition written out)
# --------------------------------------------------------------------------

def jacobi5_sweep_f32(u0: np.ndarray) -> np.ndarray:
    """One sweep in float32, grouping ``((N + S) + (W + E)) * 0.25`` on the interior."""
    u0 = np.asarray(u0, dtype=np.float32)
    u1 = u0.copy()
    n_ = u0[:-2, 1:-1]
    s_ = u0[2:, 1:-1]
    w_ = u0[1:-1, :-2]
    e_ = u0[1:-1, 2:]
    u1[1:-1, 1:-1] = ((n_ + s_) + (w_ + e_)) * np.float32(0.25)
    return u1


def jacobi5_sweep_f64(u0: np.ndarray) -> np.ndarray:
    u0 = np.asarray(u0, dtype=np.float64)
    u1 = u0.copy()
    u1[1:-1, 1:-1] = ((u0[:-2, 1:-1] + u0[2:, 1:-1]) + (u0[1:-1, :-2] + u0[1:-1, 2:])) * 0.25
    return u1


def max_update_f64(u1: np.ndarray, u0: np.ndarray) -> float:
    """``max over the interior of |(double) u1 - (double) u0|`` (sec. 5 reduction, max)."""
    return update_f64(u1, u0, "max")


def update_f64(u1: np.ndarray, u0: np.ndarray, op: str = "max") -> float:
    """Reduction of ``|(double) u1 - (double) u0|`` over the interior (sec. 5).

    ``op`` is "max", "min" or "sum"; the sum is correctly rounded (fsum).
    An interior with no points gives 0 for "max" and "sum" (the values are
    non-negative) and +inf for "min".
    """
    if u0.shape[0] < 3 or u0.shape[1] < 3:
        return math.inf if op == "min" else 0.0
    d = np.abs(u1[1:-1, 1:-1].astype(np.float64) - u0[1:-1, 1:-1].astype(np.float64))
    if op == "max":
        return float(d.max())
    if op == "min":
        return float(d.min())
    if op == "sum":
        return math.fsum(d.ravel().tolist())
    raise ValueError(op)


def jacobi5(u0: np.ndarray, sweeps: int, mode: str = "f32", op: str = "max"):
    """``sweeps`` Jacobi sweeps; returns (final grid, residual per sweep).

    The residual of a sweep is ``update_f64(new, old, op)``.
    mode "f32" reproduces float32 operation order exactly; mode "f64" runs
    the same recurrence in float64 (for error reports).
    """
    step = jacobi5_sweep_f32 if mode == "f32" else jacobi5_sweep_f64
    u = np.asarray(u0, dtype=np.float32 if mode == "f32" else np.float64)
    res = []
    for _ in range(sweeps):
        u1 = step(u)
        res.append(update_f64(u1, u, op))
        u = u1
    return u, np.array(res, dtype=np.float64)


def filter7(src: np.ndarray, w: np.ndarray, dst: np.ndarray = None) -> np.ndarray:
    """2-D stencil with a 7 x 7 filter (sec. 6, the stencil of "filter size 7").

    For every point at distance >= 3 from the edge,
    ``out[i, j] = sum over m, n in 0..6 of w[m, n] * src[i + m - 3, j + n - 3]``,
    accumulated in float32 by fused multiply-adds in the order m = 0..6 (outer),
    n = 0..6 (inner), starting from 0. Points within 3 of the edge keep the
    value of ``dst`` (of ``src`` when ``dst`` is None).
    """
    src = np.asarray(src, dtype=np.float32)
    w = np.asarray(w, dtype=np.float32).reshape(7, 7)
    out = np.array(src if dst is None else dst, dtype=np.float32, copy=True)
    H, W = src.shape
    if H < 7 or W < 7:
        return out
    s = np.zeros((H - 6, W - 6), dtype=np.float32)
    for m in range(7):
        for n in range(7):
            s = fma_f32(w[m, n], src[m:m + H - 6, n:n + W - 6], s)
    out[3:-3, 3:-3] = s
    return out


# --------------------------------------------------------------------------
# matvec and matmul (sec. 6.2 names them; definitions written out)
# --------------------------------------------------------------------------

def matvec(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    """``y[r] = sum_c A[r, c] x[c]`` in float64."""
    return np.asarray(A, np.float64) @ np.asarray(x, np.float64)


def matvec_row(A_row: np.ndarray, x: np.ndarray) -> float:
    return math.fsum((np.asarray(A_row, np.float64) * np.asarray(x, np.float64)).tolist())


def matmul(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """``C = A B`` in float64 (each float32 product exact in float64)."""
    return np.asarray(A, np.float64) @ np.asarray(B, np.float64)


def matmul_entry(A: np.ndarray, B: np.ndarray, i: int, j: int) -> float:
    """One entry of ``A B``, k ascending, exact products, correctly rounded sum."""
    return math.fsum((np.asarray(A[i, :], np.float64) * np.asarray(B[:, j], np.float64)).tolist())


def rne_bf16(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32 values.

    bfloat16 keeps the top 16 bits of the float32 pattern. Adding
    ``0x7FFF + lsb`` (lsb = bit 16) to the pattern and clearing the low 16
    bits rounds to nearest with ties to even; it carries into the exponent
    when the mantissa overflows and takes the largest finite values to
    infinity, as rounding should. NaNs are kept quiet NaNs.
    """
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (b & 0x7FFFFFFF) > 0x7F800000
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) & 0xFFFF0000) & 0xFFFFFFFF
    r = np.where(nan, (b | 0x00400000) & 0xFFFF0000, r)
    return r.astype(np.uint32).view(np.float32)


def split_bf16(x: np.ndarray):
    """(hi, lo) with ``hi = rne_bf16(x)`` and ``lo = rne_bf16(x - hi)``.

    ``x - hi`` is exact in float32: hi agrees with x in sign and exponent
    range and differs from it by at most half a bfloat16 ulp.
    """
    x = np.asarray(x, dtype=np.float32)
    hi = rne_bf16(x)
    lo = rne_bf16(x - hi)
    return hi, lo


def matmul_bf16(A, B):
    """The product of the bfloat16 roundings of A and B, in float64."""
    return matmul(rne_bf16(A), rne_bf16(B))


def matmul_split3(A, B):
    """``lo_A hi_B + hi_A lo_B + hi_A hi_B`` in float64 (the three-pass split product)."""
    ah, al = split_bf16(A)
    bh, bl = split_bf16(B)
    return matmul(al, bh) + matmul(ah, bl) + matmul(ah, bh)


def frob_rel(C, Cref) -> float:
    """Normwise relative error ``||C - Cref||_F / ||Cref||_F``."""
    C = np.asarray(C, np.float64)
    Cref = np.asarray(Cref, np.float64)
    den = np.linalg.norm(Cref)
    num = np.linalg.norm(C - Cref)
    return float(num / den) if den > 0 else float(num)
