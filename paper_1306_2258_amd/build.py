"""Builds libsas_debye.so (HIP, gfx950) in place next to this file.

    python -m paper_1306_2258_amd.build

Every HIP source is compiled with hipcc for gfx950 only.  Packed FP32
instructions are disabled at the target level (-packed-fp32-ops): the forward
recurrence is written for plain v_add_f32 / v_fmac_f32 issue.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsas_debye.so")
SOURCES = ["sas_kernels.hip", "sas_tablegrad.hip", "sas_peratom.hip", "sas_adjoint.hip", "sas_orient.hip",
           "sas_api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found (ROCm is required to build the library)")
    return path


def flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source (in parallel) and link the shared library;
    returns its path."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        cmds.append([hipcc(), *flags(), "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = jobs or min(len(cmds), os.cpu_count() or 1, 8)
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as pool:
        codes = list(pool.map(lambda c: subprocess.run(c).returncode, cmds))
    for cmd, code in zip(cmds, codes):
        if code != 0:
            raise subprocess.CalledProcessError(code, cmd)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
