"""The strip schedule of the pair kernels, checked on the CPU.

The forward and adjoint kernels decode their strip (I block, run of J blocks)
from the work-group index in closed form, and the gradient reduce walks the
strips of every row that hold an atom's J block.  ``schedule_check.cpp``
compiles the library's own schedule header for the host and compares every
one of these functions with brute-force enumeration over many sizes and
geometries (I blocks of 64 and 128 atoms, J blocks of 64..512, strips of
1..1024 J blocks), checks that every pair i < j lies in exactly one strip,
and that the launchers' geometry guard refuses J blocks that are not made of
whole I blocks (the geometry of a GPU fault the guard now prevents).
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _compiler():
    for cxx in ("g++", "c++", "clang++"):
        if shutil.which(cxx):
            return cxx
    return None


def test_strip_schedule_against_brute_force(tmp_path):
    cxx = _compiler()
    if cxx is None:
        pytest.skip("no host C++ compiler")
    inc = os.environ.get("ROCM_PATH", "/opt/rocm") + "/include"
    exe = str(tmp_path / "schedule_check")
    subprocess.check_call([cxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", inc,
                           os.path.join(HERE, "schedule_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(out.stdout)
    assert out.returncode == 0, out.stdout[-2000:]
    assert out.stdout.strip().startswith("ok")
