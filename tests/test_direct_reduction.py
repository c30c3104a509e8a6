"""CPU emulation of the direct form's reductions of t = q r / pi.

The kernel adds 1.5 * 2^21 + 1/2 to q * (r/pi) in one FP64 FMA, reads the
sum's low word as a signed integer L = v 2^31 with v = t + 1/2 (mod 2), and
evaluates w sin(pi t) = w sin(pi (|v| - 1/2)) in FP32: b = |L| 2^-31 - 1/2 by
one FMA, then b (w P)(b^2), where the pair weight w is folded into the
degree-4 polynomial's coefficients once per pair (w c_k, each rounded to
FP32).  Pairs with t <= 1/2 at every q of a chunk take the product form
instead: b = q * (r/pi) in FP64 rounded once to FP32, no reduction.  These
tests emulate each step bit for bit (the FP64 operations with exact
rationals, the FP32 steps as single roundings of exact values) and pin the
results to 40-digit sines: the one-FMA form's absolute error is that of the
exact reduction and its relative error stays below 2.5e-7 down to t = 1/4,
the smallest t the kernel sends that way (below it the conversion's 2^-25
error in b would dominate); the product form keeps the relative error below
2.5e-7 for every t <= 1/2.  Errors are in units of w.  The constants are read
from the kernel's header."""
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


def weighted_sine(b, w) -> float:
    """b (w P)(b^2) as the kernel forms it: the coefficients w c_k rounded to
    FP32 once per pair, Horner's rule, the last step an FMA into the sum."""
    wc = [f32(Fraction(float(w)) * Fraction(float(c))) for c in P]
    y = f32(b * b)
    p = fma32(y, wc[4], wc[3])
    p = fma32(p, y, wc[2])
    p = fma32(p, y, wc[1])
    p = fma32(p, y, wc[0])
    return float(fma32(b, p, f32(0.0)))


def sin_pi_t_fast(q: float, rp: float, w=f32(1.0)) -> float:
    """The one-FMA form's steps for one pair and q: w sin(pi t)."""
    magic = Fraction(MAGIC)
    s = Fraction(q) * Fraction(rp) + magic
    assert 2**21 <= s < 2**22  # the binade whose last bit is worth 2^-31
    n = round_to_multiple(s, Fraction(1, 2**31))
    lo = n & 0xFFFFFFFF
    L = lo - (1 << 32) if lo >= (1 << 31) else lo
    b = fma32(abs(f32(L)), f32(2.0**-31), f32(-0.5))
    return weighted_sine(b, w)


def sin_pi_t_product(q: float, rp: float, w=f32(1.0)) -> float:
    """The product form (t <= 1/2): b = q rp in FP64, rounded to FP32."""
    t64 = float(Fraction(q) * Fraction(rp))  # one FP64 rounding (to nearest)
    return weighted_sine(f32(t64), w)


C = [f32(_const(f"kCosPi{k}")) for k in range(6)]


def cos_pi_t_fast(q: float, rp: float) -> float:
    """The adjoint's cosine under the one-FMA reduction: cos(pi t) =
    sin(pi v) = sign(v) cos(pi b), the sign being that of the low word."""
    s = Fraction(q) * Fraction(rp) + Fraction(MAGIC)
    n = round_to_multiple(s, Fraction(1, 2**31))
    lo = n & 0xFFFFFFFF
    L = lo - (1 << 32) if lo >= (1 << 31) else lo
    b = fma32(abs(f32(L)), f32(2.0**-31), f32(-0.5))
    y = f32(b * b)
    c = fma32(y, C[5], C[4])
    for k in (3, 2, 1, 0):
        c = fma32(c, y, C[k])
    return -float(c) if lo & 0x80000000 else float(c)


def exact_cos_pi_t(q: float, rp: float) -> float:
    mpmath.mp.dps = 40
    t = Fraction(q) * Fraction(rp)
    return float(mpmath.cos(mpmath.pi * mpmath.mpf(t.numerator) / t.denominator))


@pytest.mark.parametrize("lo,hi,seed", [(0.25, 0.5, 8), (0.5, 8.0, 9), (8.0, 2.0**19, 10)])
def test_fast_reduction_cosine(lo, hi, seed):
    """The cosine's sign from the sum's low word: absolute error of the exact
    reduction's size over every half period (a wrong sign would be off by up
    to 2)."""
    rng = np.random.default_rng(seed)
    t = np.exp(rng.uniform(np.log(lo), np.log(hi), 1500))
    q = rng.uniform(1e-3, 2.0, t.size)
    worst = 0.0
    for qq, tt in zip(q, t):
        rp = float(tt / qq)
        worst = max(worst, abs(cos_pi_t_fast(float(qq), rp) - exact_cos_pi_t(float(qq), rp)))
    assert worst <= 2.5e-7


def exact_sin_pi_t(q: float, rp: float) -> float:
    mpmath.mp.dps = 40
    t = Fraction(q) * Fraction(rp)
    return float(mpmath.sin(mpmath.pi * mpmath.mpf(t.numerator) / t.denominator))


def test_constants():
    assert MAGIC == 1.5 * 2**21 + 0.5
    assert T_MIN == 0.25 and T_MAX == 2.0**19
    # the sum stays in [2^21, 2^22) over the whole range
    assert 2**21 <= MAGIC + T_MIN and MAGIC + T_MAX < 2**22


def random_weights(rng, size):
    """w = 1/r in FP32 for r from 1 to 3000 A (log-uniform)."""
    return f32(1.0) / np.exp(rng.uniform(0.0, np.log(3000.0), size)).astype(np.float32)


@pytest.mark.parametrize("lo,hi,seed", [(0.25, 0.5, 1), (0.5, 8.0, 2), (8.0, 2.0**19, 3)])
def test_fast_reduction_error_bound(lo, hi, seed):
    rng = np.random.default_rng(seed)
    t = np.exp(rng.uniform(np.log(lo), np.log(hi), 1500))
    q = rng.uniform(1e-3, 2.0, t.size)
    w = random_weights(rng, t.size)
    worst_abs = worst_rel = 0.0
    for qq, tt, ww in zip(q, t, w):
        rp = float(tt / qq)
        got, ref = sin_pi_t_fast(float(qq), rp, ww) / float(ww), exact_sin_pi_t(float(qq), rp)
        worst_abs = max(worst_abs, abs(got - ref))
        if tt < 0.5:
            worst_rel = max(worst_rel, abs(got - ref) / abs(ref))
    assert worst_abs <= 2.5e-7
    assert worst_rel <= 2.5e-7


@pytest.mark.parametrize("lo,hi,seed", [(1e-9, 1e-3, 5), (1e-3, 0.25, 6), (0.25, 0.5, 7)])
def test_product_form_error_bound(lo, hi, seed):
    """t <= 1/2 needs no reduction: the relative error holds at any small t."""
    rng = np.random.default_rng(seed)
    t = np.exp(rng.uniform(np.log(lo), np.log(hi), 1500))
    q = rng.uniform(1e-3, 2.0, t.size)
    w = random_weights(rng, t.size)
    worst = 0.0
    for qq, tt, ww in zip(q, t, w):
        rp = float(tt / qq)
        got, ref = sin_pi_t_product(float(qq), rp, ww) / float(ww), exact_sin_pi_t(float(qq), rp)
        worst = max(worst, abs(got - ref) / abs(ref))
    assert worst <= 2.5e-7


def test_zero_q_adds_nothing():
    """q = 0 (a grid's first point) gives sin = 0 exactly under both forms,
    which is why a chunk's reduction bounds come from its smallest positive q."""
    for rp in (0.01, 1.0, 317.0, 2.0**18):
        assert sin_pi_t_fast(0.0, rp, f32(0.37)) == 0.0
        assert sin_pi_t_product(0.0, rp, f32(0.37)) == 0.0


def test_integer_and_half_integer_t():
    """t on and next to integers and half-integers: the sign and the zeros."""
    for k in (1, 2, 3, 7, 100, 4097):
        for tt in (k, k + 0.5, k - 1e-6, k + 1e-6):
            q = 0.37
            rp = tt / q
            got, ref = sin_pi_t_fast(q, rp), exact_sin_pi_t(q, rp)
            assert abs(got - ref) <= 2.0e-7, (tt, got, ref)


def test_small_t_is_left_to_the_other_forms():
    """Below t = 1/4 the conversion's error in b grows relative to the sine:
    at t = 1e-3 it exceeds the bar, which is why those pairs take the product
    form (t <= 1/2 over the chunk) or the exact reduction."""
    rng = np.random.default_rng(4)
    worst = 0.0
    for tt in rng.uniform(0.9e-3, 1.1e-3, 200):
        q = 0.5
        rp = float(tt / q)
        got, ref = sin_pi_t_fast(q, rp), exact_sin_pi_t(q, rp)
        worst = max(worst, abs(got - ref) / abs(ref))
    assert worst > 1e-6
