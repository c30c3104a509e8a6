"""Comparison of a coordinate gradient with the oracle's, by norm and atom by atom.

A gradient checked only through one global 2-norm could hide a few wrong
atoms (at the edge of an I block or a strip, say) under the norm.  Every
coordinate-gradient test therefore bounds both

    ||g - g_ref||_2 / ||g_ref||_2                      (relative norm)
    max_i |g_i - g_ref,i| / max_i |g_ref,i|            (worst atom, |.| the 3-vector norm)

by the same tolerance.
"""
from __future__ import annotations

import numpy as np

# Relative tolerance of the coordinate gradient (norm and worst atom).
GTOL = 1e-5


def grad_errors(got, ref) -> tuple[float, float]:
    got = np.asarray(got, dtype=np.float64).reshape(-1, 3)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    e_norm = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    e_atom = float(np.max(np.linalg.norm(got - ref, axis=1)) / np.max(np.linalg.norm(ref, axis=1)))
    return e_norm, e_atom


def assert_grad_close(got, ref, tol: float = GTOL, what: str = "") -> tuple[float, float]:
    assert np.all(np.isfinite(got)), f"{what}: non-finite gradient"
    e_norm, e_atom = grad_errors(got, ref)
    print(f"{what} gradient: rel norm err {e_norm:.3e}, worst atom {e_atom:.3e}", flush=True)
    assert e_norm <= tol, f"{what}: relative norm error {e_norm:.3e} > {tol:g}"
    assert e_atom <= tol, f"{what}: worst-atom error {e_atom:.3e} > {tol:g}"
    return e_norm, e_atom
