"""Exhaustive CPU check of the library's host-built tables.

tests/host/table_check.cpp compiles the library's host source and checks, for
every pair state, choice and 4^8 neighbourhood, that the transition and
threshold tables send each coupled-pair move to the right threshold (equal
to the oracle's) and the right energy-change triple.  No GPU is used.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(f"{ROCM}/include/hip/hip_runtime.h"),
                    reason="needs g++ and the HIP headers")
def test_host_tables_exhaustive():
    with tempfile.TemporaryDirectory() as d:
        obj = os.path.join(d, "oracle.o")
        exe = os.path.join(d, "table_check")
        subprocess.check_call(["gcc", *[f for f in oracle.GCC_FLAGS if f != "-shared"], "-c", "-o", obj,
                               os.path.join(ROOT, "oracle", "oracle.c")])
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
                               f"-I{ROCM}/include", "-o", exe, os.path.join(ROOT, "tests", "host", "table_check.cpp"),
                               obj, f"-L{ROCM}/lib", "-lamdhip64", "-lm"])
        env = dict(os.environ, LD_LIBRARY_PATH=f"{ROCM}/lib:" + os.environ.get("LD_LIBRARY_PATH", ""))
        out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert out.returncode == 0 and out.stdout.startswith("OK"), out.stdout + out.stderr
