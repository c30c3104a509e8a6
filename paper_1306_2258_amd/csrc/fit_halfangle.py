"""Derives the FP64 coefficients of the pair set-up's half-angle sine and cosine.

The recurrence's set-up needs sin(x) and cos(x) for the half step
x = dp / 2, |x| <= pi/4 (and the quadrant-reduced seed angle, same range).
Every value derived from them is rounded to FP32 afterwards, so a relative
error far below FP32's 6e-8 suffices; with y = x^2:
  sin(x) = x + x y P(y),  P of degree 3: relative error 5e-12;
  cos(x) = 1 + y Q(y),    Q of degree 3: relative error 7e-11.
Both minimise the largest relative error of sin(x) and cos(x) on
|x| <= X = pi/4 (1 + 1e-4) by the Remez exchange, with the targets
(sin(x)/x - 1)/y and (cos(x) - 1)/y summed from their Taylor series (exact to
FP64 rounding on this range).  Run it to reproduce kHs1..kHs4 and kHc1..kHc4
in sas_device.hpp:

    python paper_1306_2258_amd/csrc/fit_halfangle.py
"""
from __future__ import annotations

import math

import numpy as np

X = math.pi / 4 * (1 + 1e-4)
Y0, Y1 = 1e-12, X * X


def series(y: np.ndarray, cos: bool) -> tuple[np.ndarray, np.ndarray]:
    """(t, f): t = (g - 1)/y and f = g for g = sin(x)/x or cos(x)."""
    t = np.zeros_like(y)
    term = np.full_like(y, -1.0 / (2.0 if cos else 6.0))
    for n in range(1, 30):
        t += term
        a, b = (2 * n + 1, 2 * n + 2) if cos else (2 * n + 2, 2 * n + 3)
        term = -term * y / (a * b)
    return t, 1.0 + y * t


def remez(cos: bool, deg: int = 3, iters: int = 60) -> tuple[np.ndarray, float]:
    """Coefficients (ascending powers of y) of the polynomial that minimises
    max |y (P(y) - t(y)) / f(y)| (the relative error of sin or cos), and that
    level."""
    n = deg + 2
    grid = Y0 + (Y1 - Y0) * (0.5 - 0.5 * np.cos(np.pi * np.linspace(0.0, 1.0, 200001)))
    tg, fg = series(grid, cos)
    wg = grid / fg  # relative error = w (P - t)
    ref = Y0 + (Y1 - Y0) * (0.5 - 0.5 * np.cos(np.pi * np.arange(n) / (n - 1)))
    coef, level = None, 0.0
    for _ in range(iters):
        tr, fr = series(ref, cos)
        wr = ref / fr
        a = np.zeros((n, n))
        for i in range(n):
            a[i, :deg + 1] = ref[i] ** np.arange(deg + 1)
            a[i, deg + 1] = -((-1) ** i) / wr[i]
        sol = np.linalg.solve(a, tr)
        coef, level = sol[:deg + 1], sol[deg + 1]
        err = wg * (np.polyval(coef[::-1], grid) - tg)
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


def check(coef: np.ndarray, cos: bool) -> float:
    """Largest relative error of the approximation on 0 < x <= X (FP64)."""
    x = np.linspace(1e-6, X, 400001)
    y = x * x
    t, f = series(y, cos)
    return float(np.max(np.abs(y * (np.polyval(coef[::-1], y) - t)) / np.abs(f)))


def main() -> None:
    for cos, name in ((False, "kHs"), (True, "kHc")):
        coef, level = remez(cos)
        print(f"{'cos' if cos else 'sin'}: minimax relative error {level:.3e} (checked {check(coef, cos):.3e})")
        for k, c in enumerate(coef):
            print(f"constexpr double {name}{k + 1} = {float(c).hex()};  // {float(c)!r}")


if __name__ == "__main__":
    main()
