"""Seeded, counter-based synthetic input generators.

This module is shared by the test suite, the benchmark and the oracle's
golden-value script. It holds no arithmetic of the loop library or of the
oracle: it only turns (seed, stream, index) into numbers.

Generator
---------
SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) is used as a counter-based hash: its 64-bit
finalizer ``mix64`` is applied to ``key + (index + 1) * GOLDEN`` where
``key = mix64(seed + stream * GOLDEN)`` and all arithmetic is modulo 2**64.

Value maps (chosen so that every value sits on a short binary grid):

* ``uniform_pm1``  : ``k = h >> 40`` (24 bits), value ``(k - 2**23) * 2**-23``
  -> multiples of 2**-23 in [-1, 1).
* ``uniform_01``   : ``k * 2**-24`` -> multiples of 2**-24 in [0, 1).
* ``normal``       : Box-Muller in float64 from two 53-bit uniforms, rounded
  to float32 (host only).
* ``int_range``    : ``lo + (h >> 11) % (hi - lo)`` (small ranges only).

Every integer-only map has a numpy implementation and a torch implementation
(CPU or GPU) that produce identical bits; the torch one lets large inputs be
generated where they will be used.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK64 = (1 << 64) - 1

__all__ = [
    "mix64", "hash_u64", "uniform_pm1", "uniform_01", "normal", "int_range",
    "uniform_pm1_torch", "uniform_01_torch", "hash_u64_torch",
]


def mix64(z: int) -> int:
    """SplitMix64 finalizer on one Python int (mod 2**64)."""
    z &= _MASK64
    z = ((z ^ (z >> 30)) * _M1) & _MASK64
    z = ((z ^ (z >> 27)) * _M2) & _MASK64
    return z ^ (z >> 31)


def _key(seed: int, stream: int) -> int:
    return mix64((seed + stream * GOLDEN) & _MASK64)


def hash_u64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Counter-based hashes h(seed, stream, i) for i in [start, start + n)."""
    key = np.uint64(_key(seed, stream))
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = key + i * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """float32 values on the 2**-23 grid in [-1, 1)."""
    k = (hash_u64(seed, stream, n, start) >> np.uint64(40)).astype(np.int64)
    return ((k - (1 << 23)).astype(np.float64) * 2.0 ** -23).astype(np.float32)


def uniform_01(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """float32 values on the 2**-24 grid in [0, 1)."""
    k = (hash_u64(seed, stream, n, start) >> np.uint64(40)).astype(np.float64)
    return (k * 2.0 ** -24).astype(np.float32)


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    """float32 standard normal values (Box-Muller in float64)."""
    h = hash_u64(seed, stream, 2 * n)
    u = (h >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u1 = 1.0 - u[0::2]          # (0, 1]
    u2 = u[1::2]
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    return z.astype(np.float32)


def int_range(seed: int, stream: int, n: int, lo: int, hi: int) -> np.ndarray:
    """int64 values in [lo, hi) (modulo map; fine for small ranges)."""
    h = hash_u64(seed, stream, n) >> np.uint64(11)
    return (h % np.uint64(hi - lo)).astype(np.int64) + lo


def uniform01_f64(seed: int, stream: int, n: int) -> np.ndarray:
    """float64 uniforms in [0, 1) with 53 random bits (host only)."""
    return (hash_u64(seed, stream, n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


# --------------------------------------------------------------------------
# torch versions (same bits). torch has no unsigned 64-bit arithmetic with
# logical shifts, so int64 two's-complement wrap-around is used and every
# right shift is followed by a mask that clears the sign-extended bits.
# --------------------------------------------------------------------------

def _to_i64(u: int) -> int:
    u &= _MASK64
    return u - (1 << 64) if u >= (1 << 63) else u


def _lsr(torch, z, s: int):
    return (z >> s) & ((1 << (64 - s)) - 1)


def hash_u64_torch(seed: int, stream: int, n: int, start: int = 0, device="cpu"):
    import torch
    key = _to_i64(_key(seed, stream))
    z = torch.arange(start + 1, start + n + 1, dtype=torch.int64, device=device)
    z = z * _to_i64(GOLDEN) + key
    z = (z ^ _lsr(torch, z, 30)) * _to_i64(_M1)
    z = (z ^ _lsr(torch, z, 27)) * _to_i64(_M2)
    z = z ^ _lsr(torch, z, 31)
    return z


def uniform_pm1_torch(seed: int, stream: int, n: int, start: int = 0, device="cpu"):
    import torch
    k = _lsr(torch, hash_u64_torch(seed, stream, n, start, device), 40)
    return ((k - (1 << 23)).to(torch.float64) * 2.0 ** -23).to(torch.float32)


def uniform_01_torch(seed: int, stream: int, n: int, start: int = 0, device="cpu"):
    import torch
    k = _lsr(torch, hash_u64_torch(seed, stream, n, start, device), 40)
    return (k.to(torch.float64) * 2.0 ** -24).to(torch.float32)


def uniform_pm1_torch_segments(seed: int, streams, lengths, align: int = 64, device="cpu",
                               chunk: int = 1 << 27):
    """Many uniform_pm1 sequences in one buffer: segment k holds
    uniform_pm1(seed, streams[k], lengths[k]) and starts at a multiple of
    `align` elements (the gap holds the same stream's next values). Returns
    (buffer, offsets). Generated in a few passes of `chunk` elements, so a
    whole workload costs tens of kernel launches, not tens per segment."""
    import torch
    lengths = np.asarray(lengths, dtype=np.int64)
    padded = (lengths + align - 1) // align * align
    offs = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(padded, out=offs[1:])
    total = int(offs[-1])
    keys = torch.tensor([_to_i64(_key(seed, int(st))) for st in streams] or [0], dtype=torch.int64, device=device)
    starts = torch.from_numpy(offs[:-1].copy()).to(device)
    seg_bounds = torch.from_numpy(offs[1:].copy()).to(device)
    out = torch.empty(total, dtype=torch.float32, device=device)
    for c0 in range(0, total, chunk):
        c1 = min(total, c0 + chunk)
        g = torch.arange(c0, c1, dtype=torch.int64, device=device)
        seg = torch.searchsorted(seg_bounds, g, right=True)
        z = (g - starts[seg] + 1) * _to_i64(GOLDEN) + keys[seg]
        z = (z ^ _lsr(torch, z, 30)) * _to_i64(_M1)
        z = (z ^ _lsr(torch, z, 27)) * _to_i64(_M2)
        z = z ^ _lsr(torch, z, 31)
        k = _lsr(torch, z, 40)
        out[c0:c1] = ((k - (1 << 23)).to(torch.float64) * 2.0 ** -23).to(torch.float32)
    return out, offs


# --------------------------------------------------------------------------
# The batched-task workload: many uneven 1-D loops with random depend edges.
# Only the recipe of the inputs (kinds, lengths, edges, values) lives here.
# --------------------------------------------------------------------------

BATCHED_KINDS = ("axpy", "sum", "matvec")


def batched_spec(seed: int, n_tasks: int, lmin: int = 8, lmax: int = 22, p_edge: float | None = None):
    """Task j: kind uniform over AXPY / SUM / MATVEC (stream 100), length
    floor(2**u) with u uniform in [lmin, lmax] (stream 101; a MATVEC of length
    L is floor(L / 256) rows (at least one) of 256 columns), and an edge i -> j
    for each i < j with probability p_edge (default 4 / (n_tasks - 1), i.e. two
    successors per task on average; stream 1000 + j).
    Returns (kinds, lengths, preds)."""
    kinds = [BATCHED_KINDS[int(k)] for k in int_range(seed, 100, n_tasks, 0, 3)]
    u = uniform01_f64(seed, 101, n_tasks)
    lens = [int(v) for v in np.floor(2.0 ** (lmin + (lmax - lmin) * u)).astype(np.int64)]
    p = p_edge if p_edge is not None else 4.0 / max(1, n_tasks - 1)
    preds = []
    for j in range(n_tasks):
        r = uniform01_f64(seed, 1000 + j, max(j, 1))[:j]
        preds.append([int(i) for i in np.nonzero(r < p)[0]])
    return kinds, lens, preds


def batched_rows(L: int) -> int:
    return max(1, L // 256)


def batched_inputs(seed: int, j: int, kind: str, L: int) -> dict:
    """Host inputs of task j: AXPY x, y (streams 10j+1, 10j+2) and a = 2.5;
    SUM x (stream 10j+1); MATVEC A (rows x 256, stream 10j+1) and x (256,
    stream 10j+2). All uniform[-1, 1) on the 2**-23 grid."""
    if kind == "axpy":
        return {"a": 2.5, "x": uniform_pm1(seed, 10 * j + 1, L), "y": uniform_pm1(seed, 10 * j + 2, L)}
    if kind == "sum":
        return {"x": uniform_pm1(seed, 10 * j + 1, L)}
    rows = batched_rows(L)
    return {"A": uniform_pm1(seed, 10 * j + 1, rows * 256).reshape(rows, 256), "x": uniform_pm1(seed, 10 * j + 2, 256)}


def batched_inputs_torch_all(seed: int, kinds, lens, device="cuda") -> list:
    """batched_inputs_torch for every task at once: the same values, as
    views into four buffers (x, y, A and the MATVEC x of all tasks), each
    task's array starting on a 256-byte boundary. A few dozen kernel
    launches for the whole workload."""
    roles = {"x": [], "y": [], "A": [], "v": []}  # (task, stream, length)
    for j, (kind, L) in enumerate(zip(kinds, lens)):
        if kind == "axpy":
            roles["x"].append((j, 10 * j + 1, L))
            roles["y"].append((j, 10 * j + 2, L))
        elif kind == "sum":
            roles["x"].append((j, 10 * j + 1, L))
        else:
            rows = batched_rows(L)
            roles["A"].append((j, 10 * j + 1, rows * 256))
            roles["v"].append((j, 10 * j + 2, 256))
    out = [dict() for _ in kinds]
    for role, items in roles.items():
        if not items:
            continue
        buf, offs = uniform_pm1_torch_segments(seed, [st for _, st, _ in items], [n for _, _, n in items],
                                               device=device)
        for k, (j, _, n) in enumerate(items):
            v = buf[int(offs[k]):int(offs[k]) + n]
            if role == "A":
                out[j]["A"] = v.reshape(-1, 256)
            else:
                out[j]["x" if role in ("x", "v") else "y"] = v
    for j, kind in enumerate(kinds):
        if kind == "axpy":
            out[j]["a"] = 2.5
    return out


def batched_inputs_torch(seed: int, j: int, kind: str, L: int, device="cuda") -> dict:
    """The same values as batched_inputs, generated by torch on `device`."""
    if kind == "axpy":
        return {"a": 2.5, "x": uniform_pm1_torch(seed, 10 * j + 1, L, device=device),
                "y": uniform_pm1_torch(seed, 10 * j + 2, L, device=device)}
    if kind == "sum":
        return {"x": uniform_pm1_torch(seed, 10 * j + 1, L, device=device)}
    rows = batched_rows(L)
    return {"A": uniform_pm1_torch(seed, 10 * j + 1, rows * 256, device=device).reshape(rows, 256),
            "x": uniform_pm1_torch(seed, 10 * j + 2, 256, device=device)}
