"""The all-cores (OpenMP) Jacobi oracle equals the serial float32-order
oracle bit for bit, grid and residuals, in several thread counts; and it
keeps the closed-form properties (linear field fixed point, impulse)."""
import numpy as np
import pytest

import synth
from oracle import bodies
from oracle import omp
from oracle.c import build as obuild


@pytest.fixture(scope="module", autouse=True)
def built():
    obuild.build()


@pytest.mark.parametrize("shape", [(5, 7), (33, 65), (130, 97), (3, 3), (2, 9)])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_omp_equals_serial_oracle(shape, threads):
    r, c = shape
    u = synth.uniform_01(5, 0, r * c).reshape(r, c)
    u[0, :] = u[-1, :] = 0
    u[:, 0] = u[:, -1] = 0
    want, wres = bodies.jacobi5(u, 7)
    got, gres, used = omp.jacobi5(u, 7, threads)
    assert used == threads
    assert np.array_equal(got, want)
    assert np.array_equal(gres, wres)


def test_omp_linear_field_fixed_point_and_impulse():
    n = 40
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    lin = (i + 2 * j).astype(np.float32)
    g, res, _ = omp.jacobi5(lin, 5, 4)
    assert np.array_equal(g, lin) and np.all(res == 0)
    imp = np.zeros((n, n), np.float32)
    imp[20, 17] = 1
    g, res, _ = omp.jacobi5(imp, 1, 4)
    assert g[20, 17] == 0 and g[19, 17] == g[21, 17] == g[20, 16] == g[20, 18] == 0.25
    assert g.sum() == 1.0 and res[0] == 1.0
