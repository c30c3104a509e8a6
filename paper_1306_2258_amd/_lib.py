"""ctypes loader for libsas_debye.so: argument marshalling only.

Every step of the computation runs in the HIP library.  If the library is
missing, or no gfx950 GPU is present, the functions here raise; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsas_debye.so")

SAS_OK = 0
STATUS_NAMES = {
    0: "SAS_OK",
    1: "SAS_ERR_INVALID_ARG",
    2: "SAS_ERR_Q_NOT_UNIFORM",
    3: "SAS_ERR_UNSUPPORTED",
    4: "SAS_ERR_WORKSPACE_TOO_SMALL",
    5: "SAS_ERR_OUT_OF_MEMORY",
    6: "SAS_ERR_HIP",
}

# Every symbol include/sas_debye.h declares, with its ctypes signature.
P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
SZ = ctypes.c_size_t
SIGNATURES = {
    "sas_version": (ctypes.c_int, []),
    "sas_create": (ctypes.c_int, [ctypes.c_int, P]),
    "sas_destroy": (None, [P]),
    "sas_last_error": (ctypes.c_char_p, []),
    "sas_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sas_q_grid_check": (ctypes.c_int, [P, I32, P, P]),
    "sas_debye_workspace_size": (SZ, [P, I64, I32, I32, ctypes.c_int]),
    "sas_debye_profile": (ctypes.c_int, [P, P, P, I64, P, I32, P, I32, P, P, SZ, P]),
    "sas_debye_profile_noalloc": (ctypes.c_int, [P, P, P, I64, P, I32, P, I32, P, P]),
    "sas_debye_workspace_size_batched": (SZ, [P, P, I32, I32, I32]),
    "sas_debye_profile_batched": (ctypes.c_int, [P, P, P, P, I32, P, I32, P, I32, P, P, SZ, P]),
    "sas_plan_create_batched": (ctypes.c_int, [P, P, P, P, I32, P, I32, P, I32, P, P, SZ, P]),
    "sas_plan_execute": (ctypes.c_int, [P, P]),
    "sas_plan_destroy": (None, [P]),
    "sas_debye_grad": (ctypes.c_int, [P, P, P, I64, P, I32, P, I32, P, P, P, P, SZ, P]),
    "sas_debye_grad_table": (ctypes.c_int, [P, P, P, I64, P, I32, P, I32, P, P, P, P, SZ, P]),
    "sas_set_variant": (ctypes.c_int, [P, I32, I32]),
    "sas_get_variant": (ctypes.c_int, [P, P, P]),
    "sas_set_form": (ctypes.c_int, [P, ctypes.c_int]),
    "sas_get_form": (ctypes.c_int, [P, P]),
    "sas_orient_degree": (I32, [ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "sas_debye_workspace_size_hybrid": (SZ, [P, I64, I32, I32, I32]),
    "sas_debye_profile_hybrid": (ctypes.c_int, [P, P, P, I64, P, I32, P, I32, ctypes.c_double, I32, P, P, SZ, P,
                                                P]),
    "sas_enable_timing": (ctypes.c_int, [P, ctypes.c_int]),
    "sas_read_timing": (ctypes.c_int, [P, P, P, P, P]),
}


class SasError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {detail}")


_lib = None


def load() -> ctypes.CDLL:
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1306_2258_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, where: str) -> None:
    if status != SAS_OK:
        detail = load().sas_last_error()
        raise SasError(status, where, detail.decode() if detail else "")
