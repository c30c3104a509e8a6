"""FP64 CPU oracle for the Debye summation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never imports it and
shares no code, headers or constants with it.

``debye_oracle.c`` is the plain definition of the Debye sum (Background
section, Eq. 2) in FP64 with compensated sums; this module only marshals
numpy arrays into it.  ``profile_numpy`` is a second, vectorised numpy
transcription used for tiny inputs in tests; ``grad_table`` is the
derivative of Eq. 2 with respect to the form-factor table, written out in
numpy; ``chi2`` holds the fit loss of the differentiation workload.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "debye_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3 -fopenmp, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_debye_profile.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int32, P, ctypes.c_int32, P, P,
                                             ctypes.c_int]
        lib.oracle_debye_profile.restype = ctypes.c_int
        lib.oracle_debye_grad.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int32, P, ctypes.c_int32, P, P,
                                          ctypes.c_int64, P, ctypes.c_int]
        lib.oracle_debye_grad.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _prep(coords, types, table, q):
    c = np.ascontiguousarray(np.asarray(coords, dtype=np.float64).reshape(-1, 3))
    t = np.ascontiguousarray(np.asarray(types, dtype=np.int32).reshape(-1))
    tab = np.ascontiguousarray(np.asarray(table, dtype=np.float64))
    qq = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1))
    if tab.ndim != 2 or tab.shape[1] != qq.shape[0]:
        raise ValueError("table must be [T, Nq] matching q")
    if c.shape[0] != t.shape[0]:
        raise ValueError("coords and types disagree on N")
    return c, t, tab, qq


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def profile(coords, types, table, q, threads: int = 0, with_abs: bool = False):
    """I(q_m) for every q_m (FP64).  Inputs are widened to FP64 exactly as given.

    With ``with_abs`` also returns A(q_m) = sum |f f sinc|, the cancellation
    measure (kappa = A / I)."""
    c, t, tab, qq = _prep(coords, types, table, q)
    I = np.zeros(qq.shape[0])
    A = np.zeros(qq.shape[0])
    rc = _load().oracle_debye_profile(_ptr(c), _ptr(t), c.shape[0], _ptr(tab), tab.shape[0], _ptr(qq), qq.shape[0],
                                      _ptr(I), _ptr(A), int(threads))
    if rc != 0:
        raise ValueError(f"oracle_debye_profile failed ({rc})")
    return (I, A) if with_abs else I


def grad(coords, types, table, q, w, atoms=None, threads: int = 0):
    """sum_m w_m dI(q_m)/dx_i for each listed atom (all atoms if None): [len, 3] FP64."""
    c, t, tab, qq = _prep(coords, types, table, q)
    ww = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1))
    if ww.shape[0] != qq.shape[0]:
        raise ValueError("w must have one weight per q")
    if atoms is None:
        at = None
        na = c.shape[0]
    else:
        at = np.ascontiguousarray(np.asarray(atoms, dtype=np.int64).reshape(-1))
        na = at.shape[0]
    g = np.zeros((na, 3))
    rc = _load().oracle_debye_grad(_ptr(c), _ptr(t), c.shape[0], _ptr(tab), tab.shape[0], _ptr(qq), qq.shape[0],
                                   _ptr(ww), _ptr(at), na, _ptr(g), int(threads))
    if rc != 0:
        raise ValueError(f"oracle_debye_grad failed ({rc})")
    return g


def profile_numpy(coords, types, table, q):
    """Eq. 2 as a full double sum over all (j, k), vectorised in numpy; tiny N only."""
    c, t, tab, qq = _prep(coords, types, table, q)
    d = c[:, None, :] - c[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    out = np.zeros(qq.shape[0])
    for m, qm in enumerate(qq):
        f = tab[t, m]
        x = qm * r
        with np.errstate(invalid="ignore", divide="ignore"):
            s = np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))
        out[m] = np.sum(f[:, None] * f[None, :] * s)
    return out


def grad_table(coords, types, table, q, w, rows: int = 512):
    """dL/dtable[t][m] = w_m dI(q_m)/df_t(q_m), FP64 [T, Nq].

    Eq. 2 is, at each q, a quadratic form in the form factors, so
        dI(q_m)/df_t(q_m) = 2 sum_{i of type t} sum_j f_{type j}(q_m) sinc(q_m r_ij)
    with j over all atoms including i (sinc(0) = 1); q values are independent.
    Written out directly in numpy (blocks of ``rows`` atoms i, all j)."""
    c, t, tab, qq = _prep(coords, types, table, q)
    ww = np.asarray(w, dtype=np.float64).reshape(-1)
    if ww.shape[0] != qq.shape[0]:
        raise ValueError("w must have one weight per q")
    n, nt = c.shape[0], tab.shape[0]
    out = np.zeros((nt, qq.shape[0]))
    for a0 in range(0, n, rows):
        a1 = min(n, a0 + rows)
        d = c[a0:a1, None, :] - c[None, :, :]
        r = np.sqrt((d * d).sum(-1))
        for m, qm in enumerate(qq):
            x = qm * r
            with np.errstate(invalid="ignore", divide="ignore"):
                s = np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))
            phi = s @ tab[t, m]
            out[:, m] += np.bincount(t[a0:a1], weights=phi, minlength=nt)
    return 2.0 * ww[None, :] * out


def chi2(I, target, rel_sigma: float = 0.01):
    """chi^2 = sum_m ((I_m - T_m) / sigma_m)^2 with sigma_m = rel_sigma * T_m, and
    its derivative w_m = dchi2/dI_m = 2 (I_m - T_m) / sigma_m^2."""
    I = np.asarray(I, dtype=np.float64)
    T = np.asarray(target, dtype=np.float64)
    sig = rel_sigma * T
    val = float(np.sum(((I - T) / sig) ** 2))
    w = 2.0 * (I - T) / sig ** 2
    return val, w
