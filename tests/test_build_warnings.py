"""The library's sources compile without warnings (CPU only).

Every HIP source is checked for both the host and the gfx950 device pass
with -Wall -Werror (syntax only, no code generated), the host-only C++
source with -Wall -Wextra -Werror. A warning here has meant a real defect
before: -Wdangling-gsl reported a reference to an element of a destroyed
temporary vector in the task engine's default-tile lookup.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2209_10643_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
INC = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hip_sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


def _hip_check(name):
    cmd = [HIPCC, "--offload-arch=gfx950", "-std=c++17", "-fsyntax-only", "-Wall", "-Werror",
           "-Wno-unused-result", "-Wno-unused-command-line-argument",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *INC, os.path.join(CSRC, name)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return name, r.returncode, r.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_hip_sources_compile_without_warnings():
    srcs = hip_sources()
    assert srcs
    with cf.ThreadPoolExecutor(min(len(srcs), 8)) as ex:
        results = list(ex.map(_hip_check, srcs))
    bad = [(n, err[-3000:]) for n, rc, err in results if rc != 0]
    assert not bad, "\n".join(f"{n}:\n{e}" for n, e in bad)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_source_compiles_without_warnings():
    for name in sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp")):
        cmd = ["g++", "-std=c++17", "-fsyntax-only", "-Wall", "-Wextra", "-Werror", *INC, os.path.join(CSRC, name)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, f"{name}:\n{r.stderr[-3000:]}"
