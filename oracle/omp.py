"""The Jacobi 5-point oracle on all host cores (OpenMP, C) -- TEST INFRASTRUCTURE.

Same loop and float32 operation order as ``bodies.jacobi5`` (sec. 6.2 2D
stencil; update ``((N + S) + (W + E)) * 0.25``, residual the max of
``|(double) u1 - (double) u0|``), run as an OpenMP ``parallel for`` with a
``reduction(max:)`` per sweep: its results equal the serial oracle's bit for
bit in any thread count (pinned by tests/test_oracle_omp.py). It exists to
time the oracle's loop on every host core; ``oracle/c/build.py`` builds it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "libjacobi5_omp.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError(f"{_LIB} is missing: build it with `python -m oracle.c.build`")
        L = C.CDLL(_LIB)
        L.jacobi5_omp.restype = C.c_int
        L.jacobi5_omp.argtypes = [C.c_void_p, C.c_void_p, C.c_long, C.c_long, C.c_int, C.c_void_p, C.c_int]
        _lib = L
    return _lib


def jacobi5(u0: np.ndarray, sweeps: int, threads: int = 0):
    """(final grid, residual per sweep, threads used) of ``sweeps`` sweeps."""
    u = np.ascontiguousarray(u0, dtype=np.float32).copy()
    tmp = np.empty_like(u)
    res = np.zeros(sweeps, np.float64)
    used = lib().jacobi5_omp(u.ctypes.data, tmp.ctypes.data, u.shape[0], u.shape[1], sweeps, res.ctypes.data,
                             int(threads))
    return u, res, used
