"""Compiles the plain C client of the library (sas_client.c) with gcc against
include/sas_debye.h, the built libsas_debye.so and the HIP runtime.

    python tests/c_client/build.py
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
BIN = os.path.join(HERE, "sas_client")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           f"-I{os.path.join(ROOT, 'include')}", os.path.join(HERE, "sas_client.c"),
           f"-L{os.path.join(ROOT, 'paper_1306_2258_amd')}", "-lsas_debye", f"-L{ROCM}/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1306_2258_amd", f"-Wl,-rpath,{ROCM}/lib", "-o", BIN]
    subprocess.check_call(cmd)
    return BIN


if __name__ == "__main__":
    print(build())
