"""Build the C parts of the oracle (test infrastructure) in-tree:

    python -m oracle.c.build

compiles jacobi5_omp.c with gcc (-O2 -fopenmp -ffp-contract=off) into
oracle/c/libjacobi5_omp.so. Only tests and the benchmark's CPU-baseline leg
load it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libjacobi5_omp.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "jacobi5_omp.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall", src,
           "-o", LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
