"""Derives the FP32 coefficients of the direct form's sine and cosine polynomials.

On |x| <= 1/2, with y = x^2:
  sin(pi x) = x * P(y), P of degree 4, minimising the largest relative error;
  cos(pi x) = Q(y),     Q of degree 5, minimising the largest absolute error
                        (cos(pi x) vanishes at the ends, where only the
                        absolute error matters for the sums it enters).
Both by the Remez exchange on y in [0, 1/4]; the coefficients are then rounded
to FP32.  Run it to reproduce kSinPi0..kSinPi4 and kCosPi0..kCosPi5 in
sas_device.hpp:

    python paper_1306_2258_amd/csrc/fit_sinpi.py
"""
from __future__ import annotations

import numpy as np

Y0, Y1 = 0.0, 0.25


def sin_target(y: np.ndarray) -> np.ndarray:
    """sin(pi sqrt(y)) / sqrt(y), with its limit pi at y = 0."""
    x = np.sqrt(y)
    safe = np.where(x > 0, x, 1.0)
    return np.where(x > 0, np.sin(np.pi * x) / safe, np.pi)


def cos_target(y: np.ndarray) -> np.ndarray:
    return np.cos(np.pi * np.sqrt(y))


def remez(target=sin_target, deg: int = 4, relative: bool = True, iters: int = 40) -> tuple[np.ndarray, float]:
    """Coefficients (ascending powers of y) and the equioscillation level."""
    n = deg + 2
    ref = (Y0 + Y1) / 2 - (Y1 - Y0) / 2 * np.cos(np.pi * np.arange(n) / (n - 1))
    grid = np.linspace(Y0, Y1, 200001)
    fg = target(grid)
    scale_g = fg if relative else np.ones_like(fg)
    coef, level = None, 0.0
    for _ in range(iters):
        # P(y_i) - f(y_i) = (-1)^i E s(y_i), s = f (relative) or 1 (absolute)
        a = np.zeros((n, n))
        for i, y in enumerate(ref):
            a[i, :deg + 1] = y ** np.arange(deg + 1)
            a[i, deg + 1] = -((-1) ** i) * (target(np.array(y)) if relative else 1.0)
        sol = np.linalg.solve(a, target(ref))
        coef, level = sol[:deg + 1], sol[deg + 1]
        err = (np.polyval(coef[::-1], grid) - fg) / scale_g
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
    x = np.linspace(-0.5, 0.5, 400001)
    coef, level = remez(sin_target, 4, True)
    c32 = coef.astype(np.float32)
    approx = x * np.polyval(c32.astype(np.float64)[::-1], x * x)
    exact = np.sin(np.pi * x)
    nz = exact != 0
    rel = np.abs(approx[nz] - exact[nz]) / np.abs(exact[nz])
    print(f"sin: minimax relative error {level:.3e}; with FP32 coefficients {rel.max():.3e}")
    for k, c in enumerate(c32):
        print(f"kSinPi{k} = {float(c).hex()}f  // {float(c)!r}")
    coef, level = remez(cos_target, 5, False)
    c32 = coef.astype(np.float32)
    err = np.abs(np.polyval(c32.astype(np.float64)[::-1], x * x) - np.cos(np.pi * x))
    print(f"cos: minimax absolute error {level:.3e}; with FP32 coefficients {err.max():.3e}")
    for k, c in enumerate(c32):
        print(f"kCosPi{k} = {float(c).hex()}f  // {float(c)!r}")


if __name__ == "__main__":
    main()
