"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

The paper prints no I(q) values (its profile figures are missing and Table 1
holds timings only), so the oracle is pinned by:
  * closed forms of Eq. 2: one atom, two atoms at exactly known sinc values,
    q = 0, regular polyhedra (pair multiplicities);
  * Eq. 1 itself: the orientational average of |sum f e^{i q.r}|^2 computed by
    Lebedev quadrature on the sphere -- an independent formula that Eq. 2 is
    the analytic integral of;
  * a 50-digit mpmath brute force (rounding of the FP64 sums);
  * invariances: rotation, translation, permutation, type relabelling, the
    bitwise power-of-two scaling r -> 2r, q -> q/2, bounds 0 < I <= (sum|f|)^2,
    the large-q limit, per-type vs per-atom tables, atom duplication;
  * the second output A(q) = sum |f f sinc| (the cancellation measure
    kappa = A / I): one and two atoms and the tetrahedron at products q r
    where sin is known exactly, A = I where no term is negative,
    |I| <= A <= (sum|f|)^2, A(0) = (sum|f(0)|)^2, and the mpmath brute force;
  * the gradient against central finite differences of the profile (by norm
    and element by element), a two-atom closed form and the exact identities
    sum_i g_i = 0, sum_i x_i x g_i = 0.
A mutation test compiles deliberately broken copies of the oracle source
(mistakes in I, in A and in the gradient) and checks that these pins reject
every one of them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W


def sinc(x):
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


# ---------------------------------------------------------------------------
# Pin checks, each written against a profile function so that the mutation
# test can run them on broken oracles too.
# ---------------------------------------------------------------------------

def pin_single_atom(profile):
    rng = np.random.default_rng(1)
    table = rng.uniform(0.5, 3.0, size=(3, 7))
    q = np.linspace(0.0, 1.2, 7)
    for t in range(3):
        I = profile(rng.normal(size=(1, 3)), np.array([t]), table, q)
        assert rel(I, table[t] ** 2) < 1e-15


def pin_two_atoms(profile):
    # r = 2 exactly; q r = pi -> sin = 0 (to 1e-16); q r = pi/2 -> sinc = 2/pi.
    coords = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    q = np.array([math.pi / 4, math.pi / 2, math.pi])
    table = np.array([[1.5, 2.0, 0.5], [3.0, 0.25, 4.0]])
    I = profile(coords, np.array([0, 1]), table, q)
    f1, f2 = table[0], table[1]
    expect = np.array([f1[0] ** 2 + f2[0] ** 2 + 2 * f1[0] * f2[0] * (2 / math.pi),
                       f1[1] ** 2 + f2[1] ** 2,
                       f1[2] ** 2 + f2[2] ** 2])
    assert rel(I, expect) < 1e-14


def pin_q_zero(profile):
    m = W.random_molecule(5, 37, 4, q0=0.0, q1=0.3)
    I = profile(m.coords, m.types, m.table, m.q)
    f0 = m.table[m.types, 0].astype(np.float64)
    assert rel(I[0], f0.sum() ** 2) < 1e-14


def _tetrahedron(a):
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    return v * a / (2 * math.sqrt(2))


def _octahedron(a):
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)
    return v * a / math.sqrt(2)


def _cube(a):
    v = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], dtype=np.float64)
    return v * a


def pin_polyhedra(profile):
    a = 3.7
    q = np.linspace(0.0, 2.5, 11)
    f = np.exp(-0.3 * q ** 2) * 6.0
    table = f[None, :]
    s = lambda d: sinc(q * d)  # noqa: E731
    cases = [
        (_tetrahedron(a), 4 * f ** 2 * (1 + 3 * s(a))),
        (_octahedron(a), 6 * f ** 2 * (1 + 4 * s(a) + s(math.sqrt(2) * a))),
        (_cube(a), 8 * f ** 2 * (1 + 3 * s(a) + 3 * s(math.sqrt(2) * a) + s(math.sqrt(3) * a))),
    ]
    for coords, expect in cases:
        I = profile(coords, np.zeros(len(coords), dtype=np.int32), table, q)
        assert rel(I, expect) < 1e-13


def eq1_quadrature(coords, types, table, q, order=131):
    """(1/4pi) * integral over the unit sphere of |sum_j f_j(q) exp(i q n.r_j)|^2 (Eq. 1)."""
    from scipy.integrate import lebedev_rule

    x, w = lebedev_rule(order)
    coords = np.asarray(coords, dtype=np.float64)
    proj = coords @ x  # [N, P]: n.r_j
    out = np.empty(len(q))
    for m, qm in enumerate(q):
        f = np.asarray(table, dtype=np.float64)[types, m]
        amp = (f[:, None] * np.exp(1j * qm * proj)).sum(axis=0)
        out[m] = float(np.sum(w * np.abs(amp) ** 2) / (4 * math.pi))
    return out


def pin_eq1(profile):
    rng = np.random.default_rng(7)
    n, t = 20, 4
    coords = rng.uniform(-5, 5, size=(n, 3))  # D <= 17.4 A
    types = rng.integers(0, t, size=n).astype(np.int32)
    q = np.linspace(0.0, 3.0, 13)  # qD <= 52 << 131
    z = np.array([1.0, 6.0, 8.0, 16.0])
    b = np.array([0.2, 0.7, 1.1, 0.4])  # per-type widths: non-separable table
    table = z[:, None] * np.exp(-b[:, None] * q[None, :] ** 2)
    I = profile(coords, types, table, q)
    assert rel(I, eq1_quadrature(coords, types, table, q)) < 1e-11


def pin_mpmath(profile):
    m = W.random_molecule(11, 12, 5, q0=0.0, q1=1.5, extent=12.0)
    I = profile(m.coords, m.types, m.table, m.q)
    exp, _ = mpmath_profile_abs(m)
    assert rel(I, exp) < 1e-13


def mpmath_profile_abs(m, dps=50):
    """Eq. 2 and A(q) = sum |f f sinc| by brute force over all (i, j) at 50 digits."""
    import mpmath

    mpmath.mp.dps = dps
    c = [[mpmath.mpf(float(v)) for v in row] for row in m.coords]
    exp, exp_abs = [], []
    for k, qm in enumerate(m.q):
        qq = mpmath.mpf(float(qm))
        tot = mpmath.mpf(0)
        tot_abs = mpmath.mpf(0)
        for i in range(m.n):
            fi = mpmath.mpf(float(m.table[m.types[i], k]))
            for j in range(m.n):
                fj = mpmath.mpf(float(m.table[m.types[j], k]))
                r = mpmath.sqrt(sum((c[i][d] - c[j][d]) ** 2 for d in range(3)))
                x = qq * r
                term = fi * fj * (1 if x == 0 else mpmath.sin(x) / x)
                tot += term
                tot_abs += abs(term)
        exp.append(float(tot))
        exp_abs.append(float(tot_abs))
    return np.array(exp), np.array(exp_abs)


def pin_invariances(profile):
    m = W.random_molecule(21, 60, 9, q0=0.0, q1=1.0, extent=25.0)
    c = m.coords.astype(np.float64)
    base = profile(c, m.types, m.table, m.q)
    rng = np.random.default_rng(3)
    qmat, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    assert rel(profile(c @ qmat.T + np.array([3.0, -7.5, 11.0]), m.types, m.table, m.q), base) < 1e-12
    perm = rng.permutation(m.n)
    assert rel(profile(c[perm], m.types[perm], m.table, m.q), base) < 1e-13
    relab = rng.permutation(m.table.shape[0])  # new id of old type t is relab[t]
    table2 = np.empty_like(m.table)
    table2[relab] = m.table
    assert rel(profile(c, relab[m.types].astype(np.int32), table2, m.q), base) < 1e-13
    # r -> 2r, q -> q/2 leaves every product q r bitwise unchanged.
    assert np.array_equal(profile(2.0 * c, m.types, m.table, m.q / 2.0), base)
    fabs = np.abs(m.table.astype(np.float64))[m.types].sum(axis=0)
    assert np.all(base > 0) and np.all(base <= fabs ** 2 * (1 + 1e-14))


def pin_large_q(profile):
    m = W.random_molecule(31, 25, 3, q0=1e4, q1=2e4, extent=10.0)
    table = np.abs(m.table.astype(np.float64)) + 1.0
    I = profile(m.coords, m.types, table, m.q)
    c = m.coords.astype(np.float64)
    d = np.sqrt(((c[:, None] - c[None]) ** 2).sum(-1))
    for k, qm in enumerate(m.q):
        f = table[m.types, k]
        diag = np.sum(f ** 2)
        off = np.abs(f[:, None] * f[None]) / np.where(d == 0, np.inf, qm * d)
        assert abs(I[k] - diag) <= off.sum() * (1 + 1e-12)


def pin_type_factoring(profile):
    m = W.random_molecule(41, 30, 6)
    per_atom = m.table.astype(np.float64)[m.types]
    I5 = profile(m.coords, m.types, m.table, m.q)
    IN = profile(m.coords, np.arange(m.n, dtype=np.int32), per_atom, m.q)
    assert rel(IN, I5) < 1e-14


def pin_duplication(profile):
    m = W.random_molecule(51, 15, 6, t=2)
    c = m.coords.astype(np.float64)
    table = m.table.astype(np.float64)
    c2 = np.vstack([c, c[:1]])
    t2 = np.concatenate([m.types, m.types[:1]]).astype(np.int32)
    table3 = np.vstack([table, 2.0 * table[m.types[0]][None]])
    t3 = m.types.copy()
    t3[0] = table.shape[0]
    assert rel(profile(c2, t2, table, m.q), profile(c, t3, table3, m.q)) < 1e-13


PINS = [pin_single_atom, pin_two_atoms, pin_q_zero, pin_polyhedra, pin_eq1, pin_mpmath, pin_invariances,
        pin_large_q, pin_type_factoring, pin_duplication]


# ---------------------------------------------------------------------------
# Pins of the second output A(q) = sum_k sum_j |f_k f_j sinc(q r_jk)| (the
# cancellation measure kappa = A / I).  Each takes profile_abs(coords, types,
# table, q) -> (I, A).  Closed forms use products q r at which sin is known
# exactly (multiples of pi/2), so no expected value re-calls a sine.
# ---------------------------------------------------------------------------

def apin_single_atom(profile_abs):
    # A = f^2, also for negative form factors (the diagonal's |f f|)
    table = np.array([[-1.5, 2.0, -0.25, 0.75]])
    q = np.array([0.0, 0.4, 1.3, 2.9])
    _, A = profile_abs(np.array([[0.3, -1.0, 2.0]]), np.array([0]), table, q)
    assert rel(A, table[0] ** 2) < 1e-15


def apin_two_atoms(profile_abs):
    # r = 2 exactly: q r = pi/2, 3pi/2, 5pi/2, 7pi/2, pi and 0, where sinc is
    # 2/pi, -2/(3pi), 2/(5pi), -2/(7pi), 0 (to 1e-16) and 1; form-factor
    # products of both signs
    coords = np.array([[0.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    q = np.array([0.0, math.pi / 4, math.pi / 2, 3 * math.pi / 4, 5 * math.pi / 4, 7 * math.pi / 4])
    s = np.array([1.0, 2 / math.pi, 0.0, -2 / (3 * math.pi), 2 / (5 * math.pi), -2 / (7 * math.pi)])
    table = np.array([[1.5, -2.0, 0.5, 3.0, -1.25, 0.8], [-3.0, 0.25, 4.0, 1.5, -2.0, 2.5]])
    I, A = profile_abs(coords, np.array([0, 1]), table, q)
    f1, f2 = table[0], table[1]
    assert rel(A, f1 ** 2 + f2 ** 2 + 2 * np.abs(f1 * f2 * s)) < 1e-14
    assert rel(I, f1 ** 2 + f2 ** 2 + 2 * f1 * f2 * s) < 1e-14


def apin_tetrahedron(profile_abs):
    # one type, edge a: A = 4 f^2 (1 + 3 |s(a)|); q a = 3pi/2 and 7pi/2 make s < 0
    a = 3.7
    q = np.array([0.0, 0.5 * math.pi / a, 1.5 * math.pi / a, 3.5 * math.pi / a])
    s = np.array([1.0, 2 / math.pi, -2 / (3 * math.pi), -2 / (7 * math.pi)])
    f = np.array([6.0, -5.5, 4.0, 2.5])
    I, A = profile_abs(_tetrahedron(a), np.zeros(4, dtype=np.int32), f[None, :], q)
    assert rel(A, 4 * f ** 2 * (1 + 3 * np.abs(s))) < 1e-13
    assert rel(I, 4 * f ** 2 * (1 + 3 * s)) < 1e-13


def apin_equals_profile_when_no_term_is_negative(profile_abs):
    # positive form factors and q D < pi: every sinc > 0, so A = I
    m = W.random_molecule(91, 40, 9, q0=0.0, q1=0.3, extent=8.0)
    c = m.coords.astype(np.float64)
    d = np.sqrt(((c[:, None] - c[None]) ** 2).sum(-1)).max()
    assert m.q[-1] * d < math.pi and np.all(m.table > 0)
    I, A = profile_abs(m.coords, m.types, m.table, m.q)
    assert rel(A, I) < 1e-14


def apin_bounds_and_q_zero(profile_abs):
    # |I| <= A <= (sum |f|)^2 everywhere, A(0) = (sum |f(0)|)^2, and A > I
    # where terms cancel (form factors of both signs, q D up to ~60)
    m = W.random_molecule(93, 50, 12, t=3, q0=0.0, q1=3.0, extent=20.0)
    table = m.table.astype(np.float64) * np.array([1.0, -1.0, 0.5])[:, None]
    I, A = profile_abs(m.coords, m.types, table, m.q)
    fabs = np.abs(table)[m.types].sum(axis=0)
    assert np.all(np.abs(I) <= A * (1 + 1e-14))
    assert np.all(A <= fabs ** 2 * (1 + 1e-14))
    assert rel(A[0], fabs[0] ** 2) < 1e-14
    assert np.all(A[1:] > np.abs(I[1:]) * (1 + 1e-3))


def apin_mpmath(profile_abs):
    m = W.random_molecule(13, 10, 4, q0=0.0, q1=2.5, extent=10.0)
    table = m.table.astype(np.float64)
    table[1] *= -1.0
    m.table = table
    I, A = profile_abs(m.coords, m.types, table, m.q)
    exp_I, exp_A = mpmath_profile_abs(m)
    assert rel(I, exp_I) < 1e-13
    assert rel(A, exp_A) < 1e-13


APINS = [apin_single_atom, apin_two_atoms, apin_tetrahedron, apin_equals_profile_when_no_term_is_negative,
         apin_bounds_and_q_zero, apin_mpmath]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_profile_pin(pin):
    pin(oracle.profile)


def _oracle_profile_abs(coords, types, table, q):
    return oracle.profile(coords, types, table, q, with_abs=True)


@pytest.mark.parametrize("pin", APINS, ids=[p.__name__ for p in APINS])
def test_oracle_abs_pin(pin):
    pin(_oracle_profile_abs)


def test_numpy_transcription_matches_c_oracle():
    m = W.random_molecule(61, 45, 8)
    assert rel(oracle.profile_numpy(m.coords, m.types, m.table, m.q),
               oracle.profile(m.coords, m.types, m.table, m.q)) < 1e-14


def test_oracle_thread_count_independent():
    m = W.random_molecule(71, 300, 6)
    a = oracle.profile(m.coords, m.types, m.table, m.q, threads=1)
    b = oracle.profile(m.coords, m.types, m.table, m.q, threads=3)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Gradient pins
# ---------------------------------------------------------------------------

def _grad_case():
    m = W.random_molecule(81, 18, 7, q0=0.0, q1=1.2, extent=9.0)
    rng = np.random.default_rng(5)
    w = rng.normal(size=len(m.q))
    return m.coords.astype(np.float64), m.types, m.table.astype(np.float64), m.q, w


# Each gradient pin takes grad(coords, types, table, q, w, atoms=None) and the
# (pinned) profile oracle, so that the mutation test can run them on broken
# gradient oracles too.

def gpin_central_differences(grad, profile):
    """Every coordinate of a small two-type molecule against central
    differences of the pinned profile oracle (h = 1e-5 A)."""
    c, t, tab, q, w = _grad_case()
    g = grad(c, t, tab, q, w)
    h = 1e-5
    num = np.zeros_like(c)
    for i in range(c.shape[0]):
        for d in range(3):
            cp = c.copy()
            cm = c.copy()
            cp[i, d] += h
            cm[i, d] -= h
            num[i, d] = (w @ profile(cp, t, tab, q) - w @ profile(cm, t, tab, q)) / (2 * h)
    assert np.linalg.norm(g - num) / np.linalg.norm(num) < 1e-7
    # element by element as well: no atom hides under the norm
    assert np.max(np.abs(g - num)) < 1e-6 * np.max(np.abs(num))


def gpin_identities(grad, profile):
    """Translation and rotation invariance of Eq. 2: the forces and their
    torques sum to zero."""
    c, t, tab, q, w = _grad_case()
    g = grad(c, t, tab, q, w)
    scale = np.abs(g).sum()
    assert np.abs(g.sum(axis=0)).max() < 1e-12 * scale
    torque = np.cross(c, g).sum(axis=0)
    assert np.abs(torque).max() < 1e-12 * scale * np.abs(c).max()


def gpin_q_zero_and_coincident_atoms_are_zero(grad, profile):
    """I(0) does not depend on the positions, and the derivative of sinc
    vanishes at 0: q = 0 weights and coincident atoms give no force."""
    c = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 2.0, 0.5]])
    tab = np.array([[2.0, 1.0]])
    q = np.array([0.0, 0.7])
    g = grad(c, np.zeros(3, dtype=np.int32), tab, q, np.array([1.0, 0.0]))
    assert np.all(g == 0.0)
    g2 = grad(c[:2], np.zeros(2, dtype=np.int32), tab, q, np.array([0.0, 1.0]))
    assert np.all(g2 == 0.0)


def gpin_two_atoms_closed_form(grad, profile):
    """Two atoms along x at r = 2 with q r = pi/2 (sin = 1, cos = 0): the
    derivative of 2 f1 f2 sin(q r)/(q r) along the axis is
    2 f1 f2 (cos(q r)/r - sin(q r)/(q r^2)) = -2 f1 f2 / (q r^2)."""
    c = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    q = np.array([math.pi / 4])
    tab = np.array([[1.5], [-2.5]])
    g = grad(c, np.array([0, 1]), tab, q, np.array([1.0]))
    d = -2.0 * 1.5 * -2.5 / (q[0] * 4.0)  # dI/dr
    # atom 1 moves away from atom 0 along +x: dI/dx_1 = dI/dr, dI/dx_0 = -dI/dr
    assert rel(g[:, 0], np.array([-d, d])) < 1e-14
    assert np.all(g[:, 1:] == 0.0)


GPINS = [gpin_central_differences, gpin_identities, gpin_q_zero_and_coincident_atoms_are_zero,
         gpin_two_atoms_closed_form]


@pytest.mark.parametrize("pin", GPINS, ids=[p.__name__ for p in GPINS])
def test_oracle_grad_pin(pin):
    pin(oracle.grad, oracle.profile)


def test_grad_atom_subset_matches_full():
    c, t, tab, q, w = _grad_case()
    g = oracle.grad(c, t, tab, q, w)
    sub = np.array([3, 0, 17, 9])
    assert np.array_equal(oracle.grad(c, t, tab, q, w, atoms=sub), g[sub])


def test_chi2_weights_are_the_derivative():
    rng = np.random.default_rng(9)
    T = rng.uniform(1, 2, size=6)
    I = T * (1 + 0.03 * rng.normal(size=6))
    val, w = oracle.chi2(I, T)
    h = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        num = (oracle.chi2(I + e, T)[0] - oracle.chi2(I - e, T)[0]) / (2 * h)
        assert abs(num - w[k]) <= 1e-6 * abs(w).max()


# ---------------------------------------------------------------------------
# Table-gradient pins
# ---------------------------------------------------------------------------

def _table_case():
    m = W.random_molecule(83, 11, 6, t=3, q0=0.0, q1=1.1, extent=8.0, widths=[0.4, 0.9, 1.5])
    w = np.random.default_rng(6).normal(size=len(m.q))
    return m.coords.astype(np.float64), m.types, m.table.astype(np.float64), m.q, w


def test_grad_table_vs_central_differences_of_the_c_oracle():
    """At each q Eq. 2 is quadratic in the table, so a central difference of
    the C oracle's profile is exact up to rounding: it pins the numpy
    derivative to an independent code path."""
    c, t, tab, q, w = _table_case()
    g = oracle.grad_table(c, t, tab, q, w)
    h = 1e-3
    num = np.zeros_like(tab)
    for a in range(tab.shape[0]):
        for m in range(tab.shape[1]):
            tp = tab.copy()
            tm = tab.copy()
            tp[a, m] += h
            tm[a, m] -= h
            dI = oracle.profile(c, t, tp, q)[m] - oracle.profile(c, t, tm, q)[m]
            num[a, m] = w[m] * dI / (2 * h)
    assert np.max(np.abs(g - num)) <= 1e-9 * np.max(np.abs(num))


def test_grad_table_euler_identity_and_special_cases():
    c, t, tab, q, w = _table_case()
    ones = np.ones(len(q))
    g = oracle.grad_table(c, t, tab, q, ones)
    # homogeneous of degree 2: sum_t f_t dI/df_t = 2 I
    assert rel((tab * g).sum(axis=0), 2.0 * oracle.profile(c, t, tab, q)) < 1e-12
    # q = 0: dI/df_t = 2 n_t sum_b n_b f_b
    n_t = np.bincount(t, minlength=tab.shape[0]).astype(np.float64)
    assert q[0] == 0.0
    assert rel(g[:, 0], 2.0 * n_t * (n_t @ tab[:, 0])) < 1e-13
    # one atom: dI/df = 2 f for its type, 0 for the others
    g1 = oracle.grad_table(c[:1], t[:1], tab, q, ones)
    assert rel(g1[t[0]], 2.0 * tab[t[0]]) < 1e-15
    assert np.all(np.delete(g1, t[0], axis=0) == 0.0)
    # the weights scale each q column
    assert rel(oracle.grad_table(c, t, tab, q, w), g * w[None, :]) < 1e-15


# ---------------------------------------------------------------------------
# Mutation test: plausible mistakes planted in copies of the oracle's C source
# (on the CPU) must each be caught by at least one pin.
# ---------------------------------------------------------------------------

# Mistakes in the profile I(q) (caught by PINS), in A(q) (caught by APINS)
# and in the gradient (caught by GPINS).
MUTANTS = {
    "no_doubling": ("double term = 2.0 * fk[m]", "double term = 1.0 * fk[m]"),
    "no_diagonal": ("neu_add(&tot, f * f);", "(void)0;"),
    "sinc0_is_zero": ("return x == 0.0 ? 1.0 : sin(x) / x;", "return x == 0.0 ? 0.0 : sin(x) / x;"),
    "wrong_partner_type": ("const double* fj = table + (int64_t)types[j] * nq;\n        for (int32_t m = 0; m < nq; ++m) {\n          double term",
                           "const double* fj = table + (int64_t)types[k] * nq;\n        for (int32_t m = 0; m < nq; ++m) {\n          double term"),
    "q_off_by_one": ("sinc(q[m] * r)", "sinc(q[m > 0 ? m - 1 : 0] * r)"),
    "dropped_dz": ("sqrt(dx * dx + dy * dy + dz * dz);\n        const double* fj",
                   "sqrt(dx * dx + dy * dy);\n        const double* fj"),
    "transposed_table": ("double f = table[(int64_t)types[k] * nq + m];", "double f = table[(int64_t)m * t + types[k] % t];"),
}
ABS_MUTANTS = {
    "abs_dropped": ("neu_add(&sA[m], fabs(term));", "neu_add(&sA[m], term);"),
    "abs_no_diagonal": ("neu_add(&tabs, f * f);", "(void)0;"),
    "abs_of_sinc_only": ("neu_add(&sA[m], fabs(term));", "neu_add(&sA[m], 2.0 * fk[m] * fj[m] * fabs(sinc(q[m] * r)));"),
    "abs_not_doubled": ("neu_add(&sA[m], fabs(term));", "neu_add(&sA[m], 0.5 * fabs(term));"),
}
GRAD_MUTANTS = {
    "grad_no_sine_term": ("double dsinc_dr = cos(x) / r - sin(x) / (q[m] * r * r);", "double dsinc_dr = cos(x) / r;"),
    "grad_sign": ("double dsinc_dr = cos(x) / r - sin(x) / (q[m] * r * r);",
                  "double dsinc_dr = sin(x) / (q[m] * r * r) - cos(x) / r;"),
    "grad_no_factor_two": ("neu_add(&dsum, 2.0 * w[m]", "neu_add(&dsum, 1.0 * w[m]"),
    "grad_partner_type": ("const double* fj = table + (int64_t)types[j] * nq;\n      neu_t dsum",
                          "const double* fj = table + (int64_t)types[i] * nq;\n      neu_t dsum"),
    "grad_not_unit_direction": ("double g = neu_val(&dsum) / r;", "double g = neu_val(&dsum);"),
    "grad_q_zero_kept": ("if (q[m] == 0.0) continue;", "(void)0;"),
    "grad_dropped_dz": ("neu_add(&gz, g * dz);", "neu_add(&gz, g * dy);"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "debye_oracle.c")).read()
    assert old in src, f"mutation anchor for {name} not found"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new, 1))
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", str(path), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    lib.oracle_debye_profile.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int32, P, ctypes.c_int32, P, P, ctypes.c_int]
    lib.oracle_debye_grad.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int32, P, ctypes.c_int32, P, P,
                                      ctypes.c_int64, P, ctypes.c_int]

    def arrays(coords, types, table, q):
        return (np.ascontiguousarray(np.asarray(coords, dtype=np.float64).reshape(-1, 3)),
                np.ascontiguousarray(np.asarray(types, dtype=np.int32)),
                np.ascontiguousarray(np.asarray(table, dtype=np.float64)),
                np.ascontiguousarray(np.asarray(q, dtype=np.float64)))

    def profile_abs(coords, types, table, q):
        c, t, tab, qq = arrays(coords, types, table, q)
        out = np.zeros(len(qq))
        a = np.zeros(len(qq))
        lib.oracle_debye_profile(c.ctypes.data, t.ctypes.data, c.shape[0], tab.ctypes.data, tab.shape[0],
                                 qq.ctypes.data, len(qq), out.ctypes.data, a.ctypes.data, 1)
        return out, a

    def profile(coords, types, table, q):
        return profile_abs(coords, types, table, q)[0]

    def grad(coords, types, table, q, w, atoms=None):
        c, t, tab, qq = arrays(coords, types, table, q)
        ww = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        assert atoms is None
        g = np.zeros((c.shape[0], 3))
        lib.oracle_debye_grad(c.ctypes.data, t.ctypes.data, c.shape[0], tab.ctypes.data, tab.shape[0],
                              qq.ctypes.data, len(qq), ww.ctypes.data, None, c.shape[0], g.ctypes.data, 1)
        return g

    return profile, profile_abs, grad


def _caught(checks):
    caught = []
    for name, fn in checks:
        try:
            fn()
        except AssertionError:
            caught.append(name)
    return caught


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    profile, _, _ = _build_mutant(tmp_path, name, old, new)
    checks = [(pin.__name__, lambda pin=pin: pin(profile)) for pin in PINS if pin is not pin_mpmath]
    assert _caught(checks), f"no pin caught mutant {name}"  # (mpmath: slow, redundant for these)


@pytest.mark.parametrize("name", sorted(ABS_MUTANTS))
def test_abs_pins_reject_mutant(tmp_path, name):
    old, new = ABS_MUTANTS[name]
    profile, profile_abs, _ = _build_mutant(tmp_path, name, old, new)
    checks = [(pin.__name__, lambda pin=pin: pin(profile_abs)) for pin in APINS if pin is not apin_mpmath]
    assert _caught(checks), f"no A(q) pin caught mutant {name}"
    # the mistakes are in A only: the profile pins still pass
    assert not _caught([(pin.__name__, lambda pin=pin: pin(profile)) for pin in PINS if pin is not pin_mpmath])


@pytest.mark.parametrize("name", sorted(GRAD_MUTANTS))
def test_grad_pins_reject_mutant(tmp_path, name):
    old, new = GRAD_MUTANTS[name]
    _, _, grad = _build_mutant(tmp_path, name, old, new)
    checks = [(pin.__name__, lambda pin=pin: pin(grad, oracle.profile)) for pin in GPINS]
    assert _caught(checks), f"no gradient pin caught mutant {name}"
