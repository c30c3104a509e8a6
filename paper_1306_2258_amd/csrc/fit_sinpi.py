"""Derives the FP32 coefficients of the direct form's sine polynomial.

sin(pi x) = x * P(x^2) on |x| <= 1/2, P of degree 4, chosen to minimise the
largest relative error (Remez exchange on y = x^2 in [0, 1/4]); the
coefficients are then rounded to FP32.  Run it to reproduce the constants
kSinPi0..kSinPi4 in sas_device.hpp:

    python paper_1306_2258_amd/csrc/fit_sinpi.py
"""
from __future__ import annotations

import numpy as np

DEG = 4
Y0, Y1 = 0.0, 0.25


def target(y: np.ndarray) -> np.ndarray:
    """sin(pi sqrt(y)) / sqrt(y), with its limit pi at y = 0."""
    x = np.sqrt(y)
    safe = np.where(x > 0, x, 1.0)
    return np.where(x > 0, np.sin(np.pi * x) / safe, np.pi)


def remez(iters: int = 40) -> tuple[np.ndarray, float]:
    n = DEG + 2
    ref = (Y0 + Y1) / 2 - (Y1 - Y0) / 2 * np.cos(np.pi * np.arange(n) / (n - 1))
    grid = np.linspace(Y0, Y1, 200001)
    fg = target(grid)
    coef, level = None, 0.0
    for _ in range(iters):
        # P(y_i) - f(y_i) = (-1)^i E f(y_i): equioscillating relative error
        a = np.zeros((n, n))
        for i, y in enumerate(ref):
            a[i, :DEG + 1] = y ** np.arange(DEG + 1)
            a[i, DEG + 1] = -((-1) ** i) * target(np.array(y))
        sol = np.linalg.solve(a, target(ref))
        coef, level = sol[:DEG + 1], sol[DEG + 1]
        err = (np.polyval(coef[::-1], grid) - fg) / fg
        # new reference: one extremum per sign run of the error
        runs, start = [], 0
        sgn = np.sign(err)
        for i in range(1, len(grid) + 1):
            if i == len(grid) or sgn[i] != sgn[start]:
                runs.append(start + int(np.argmax(np.abs(err[start:i]))))
                start = i
        while len(runs) > n:
            runs.pop(0 if abs(err[runs[0]]) < abs(err[runs[-1]]) else -1)
        if len(runs) == n:
            ref = grid[runs]
    return coef, abs(level)


def main() -> None:
    coef, level = remez()
    c32 = coef.astype(np.float32)
    x = np.linspace(-0.5, 0.5, 400001)
    approx = x * np.polyval(c32.astype(np.float64)[::-1], x * x)
    exact = np.sin(np.pi * x)
    nz = exact != 0
    rel = np.abs(approx[nz] - exact[nz]) / np.abs(exact[nz])
    print(f"minimax relative error {level:.3e}; with FP32 coefficients {rel.max():.3e}")
    for k, c in enumerate(c32):
        print(f"kSinPi{k} = {float(c).hex()}f  // {float(c)!r}")


if __name__ == "__main__":
    main()
