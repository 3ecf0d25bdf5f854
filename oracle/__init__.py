"""CPU oracle for the UPIR data-parallel loop library -- TEST INFRASTRUCTURE.

This package is the plain, slow, obviously correct reference that the HIP
path is checked against. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the library itself never does,
and this package imports nothing from the library. The two share no code;
only the seeded input generators (package ``synth``) feed both.

Every function executes a loop as its *serial elision*: the parallel
annotations removed and iterations taken in index order, in float64 unless a
function says it reproduces float32 operation order. Each function cites the
passage of the UPIR paper (Wang, Yi, Yan, arXiv 2209.10643) it follows.

Modules
-------
loops    canonical loop trip counts, collapse, worksharing owner maps (sec. 3.2)
bodies   AXPY, sum, Jacobi 5-point, matvec, matmul and BF16 splitting (sec. 6.2)
reduce   reduction operators (sec. 5)
tasks    depend -> task graph, index-order task execution, token chain (sec. 3.3)
mlp      schedule cost-model MLP forward / backward / Adam in float64
         (an extension with no passage in the paper)

Parity status: every function is pinned by tests under ``tests/`` marked
``not gpu`` (closed forms, brute force, published test vectors, invariants),
except where a module header says "parity unpinned".
"""
from . import loops, bodies, reduce, tasks, mlp  # noqa: F401
