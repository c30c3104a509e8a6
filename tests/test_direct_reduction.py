"""CPU emulation of the direct form's one-FMA reduction of t = q r / pi.

The kernel adds 1.5 * 2^21 + 1/2 to q * (r/pi) in one FP64 FMA, reads the
sum's low word as a signed integer L = v 2^31 with v = t + 1/2 (mod 2), and
evaluates sin(pi t) = sin(pi (|v| - 1/2)) in FP32: b = |L| 2^-31 - 1/2 by one
FMA, then b P(b^2) with the degree-4 polynomial of the exact form.  These
tests emulate each step bit for bit (the FP64 FMA with exact rationals, the
FP32 steps as single roundings of exact values) and pin the result to
40-digit sines: the absolute error is that of the exact reduction, and the
relative error stays below 2.5e-7 down to t = 1/4, the smallest t the kernel
sends this way (below it the conversion's 2^-25 error in b would dominate).
The constants are read from the kernel's header."""
from __future__ import annotations

import os
import re
from fractions import Fraction

import mpmath
import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1306_2258_amd", "csrc")
SRC = open(os.path.join(CSRC, "sas_device.hpp")).read()
f32 = np.float32


def _const(name):
    m = re.search(r"\b" + name + r" = (-?0x[0-9a-f]+(?:\.[0-9a-f]*)?p[+-]?\d+)f?(?: \+ ([0-9.]+))?", SRC)
    assert m, name
    v = float.fromhex(m.group(1))
    return v + float(m.group(2)) if m.group(2) else v


MAGIC = _const("kHalfMagic")
T_MIN = _const("kFracMinT")
T_MAX = _const("kFracMaxT")
P = [f32(_const(f"kSinPi{k}")) for k in range(5)]


def fma32(a, b, c):
    """FP32 FMA: the exact value a*b + c rounded once to FP32."""
    return f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def round_to_multiple(x: Fraction, ulp: Fraction) -> int:
    """x / ulp rounded to the nearest integer, ties to even (FP64 rounding of
    a sum whose exponent fixes the last bit's weight at ulp)."""
    s = x / ulp
    fl = s.numerator // s.denominator
    rem = s - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2):
        fl += 1
    return fl


def sin_pi_t_fast(q: float, rp: float) -> float:
    """The kernel's steps for one pair and q (weight 1)."""
    magic = Fraction(MAGIC)
    s = Fraction(q) * Fraction(rp) + magic
    assert 2**21 <= s < 2**22  # the binade whose last bit is worth 2^-31
    n = round_to_multiple(s, Fraction(1, 2**31))
    lo = n & 0xFFFFFFFF
    L = lo - (1 << 32) if lo >= (1 << 31) else lo
    b = fma32(abs(f32(L)), f32(2.0**-31), f32(-0.5))
    y = f32(b * b)
    p = fma32(y, P[4], P[3])
    p = fma32(p, y, P[2])
    p = fma32(p, y, P[1])
    p = fma32(p, y, P[0])
    return float(fma32(f32(b * f32(1.0)), p, f32(0.0)))


def exact_sin_pi_t(q: float, rp: float) -> float:
    mpmath.mp.dps = 40
    t = Fraction(q) * Fraction(rp)
    return float(mpmath.sin(mpmath.pi * mpmath.mpf(t.numerator) / t.denominator))


def test_constants():
    assert MAGIC == 1.5 * 2**21 + 0.5
    assert T_MIN == 0.25 and T_MAX == 2.0**19
    # the sum stays in [2^21, 2^22) over the whole range
    assert 2**21 <= MAGIC + T_MIN and MAGIC + T_MAX < 2**22


@pytest.mark.parametrize("lo,hi,seed", [(0.25, 0.5, 1), (0.5, 8.0, 2), (8.0, 2.0**19, 3)])
def test_fast_reduction_error_bound(lo, hi, seed):
    rng = np.random.default_rng(seed)
    t = np.exp(rng.uniform(np.log(lo), np.log(hi), 1500))
    q = rng.uniform(1e-3, 2.0, t.size)
    worst_abs = worst_rel = 0.0
    for qq, tt in zip(q, t):
        rp = float(tt / qq)
        got, ref = sin_pi_t_fast(float(qq), rp), exact_sin_pi_t(float(qq), rp)
        worst_abs = max(worst_abs, abs(got - ref))
        if tt < 0.5:
            worst_rel = max(worst_rel, abs(got - ref) / abs(ref))
    assert worst_abs <= 2.0e-7
    assert worst_rel <= 2.5e-7


def test_integer_and_half_integer_t():
    """t on and next to integers and half-integers: the sign and the zeros."""
    for k in (1, 2, 3, 7, 100, 4097):
        for tt in (k, k + 0.5, k - 1e-6, k + 1e-6):
            q = 0.37
            rp = tt / q
            got, ref = sin_pi_t_fast(q, rp), exact_sin_pi_t(q, rp)
            assert abs(got - ref) <= 2.0e-7, (tt, got, ref)


def test_small_t_is_left_to_the_exact_form():
    """Below t = 1/4 the conversion's error in b grows relative to the sine:
    at t = 1e-3 it exceeds the bar, which is why those pairs are reduced
    exactly."""
    rng = np.random.default_rng(4)
    worst = 0.0
    for tt in rng.uniform(0.9e-3, 1.1e-3, 200):
        q = 0.5
        rp = float(tt / q)
        got, ref = sin_pi_t_fast(q, rp), exact_sin_pi_t(q, rp)
        worst = max(worst, abs(got - ref) / abs(ref))
    assert worst > 1e-6
