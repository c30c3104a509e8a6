"""Checks of the seeded synthetic inputs (shapes, recipes, determinism)."""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads as W


def _min_dist(c):
    from scipy.spatial import cKDTree

    d, _ = cKDTree(c).query(c, k=2)
    return float(d[:, 1].min())


def test_ellipsoid_1k():
    m = W.ellipsoid_1k()
    assert m.coords.shape == (1000, 3) and m.coords.dtype == np.float32
    assert m.types.dtype == np.int32 and m.types.min() >= 0 and m.types.max() < 5
    assert m.table.shape == (5, 64) and m.table.dtype == np.float32
    assert m.q.dtype == np.float64 and m.q[0] == 0.0 and m.q[-1] == 0.5 and len(m.q) == 64
    e = (m.coords.astype(np.float64) / np.array([15.0, 12.0, 10.0])) ** 2
    assert np.all(e.sum(1) <= 1.0 + 1e-6)
    # f_t(0) = Z_t exactly
    assert np.array_equal(m.table[:, 0], np.array(W.TYPE_Z, dtype=np.float32))


def test_type_frequencies_match_recipe():
    m = W.dna_rod_50k()
    counts = np.bincount(m.types, minlength=5).astype(np.float64)
    expect = np.array(W.TYPE_PROBS) * m.n
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    assert chi2 < 20.5  # p ~ 4e-4 for 4 degrees of freedom


def test_globular_min_separation_and_radius():
    m = W.globular_10k()
    c = m.coords.astype(np.float64)
    assert m.n == 10000
    assert np.sqrt((c ** 2).sum(1)).max() <= 30.0 + 1e-4
    assert _min_dist(c) >= 1.0 - 1e-5
    assert len(m.q) == 100 and m.q[-1] == 1.0


def test_rod_geometry():
    m = W.dna_rod_50k()
    c = m.coords.astype(np.float64)
    assert m.n == 50000 and len(m.q) == 200
    length = c[:, 2].max() - c[:, 2].min()
    assert 3390 < length < 3420
    assert abs(c[:, 2].mean()) < 5.0
    rad = np.sqrt(c[:, 0] ** 2 + c[:, 1] ** 2)
    assert np.sum(rad < 4.0) >= 10000  # the core cylinder


def test_lattice_20k():
    m = W.lattice_20k()
    c = m.coords.astype(np.float64)
    assert m.n == 20000 and m.table.shape == (1, 100)
    assert _min_dist(c) >= 3.2 - 1e-4
    ext = c.max(0) - c.min(0)
    assert np.all(ext < np.array([76, 76, 228]))
    assert m.extra["target_coords"].shape == (20000, 3)


def test_ensemble_sizes_and_offsets():
    sizes = W.ensemble_sizes()
    assert len(sizes) == 256 and sizes.min() >= 500 and sizes.max() <= 8000
    assert abs(np.log(sizes).mean() - 0.5 * (math.log(500) + math.log(8000))) < 0.15
    assert W.globular_radius(10000) == 30.0 or abs(W.globular_radius(10000) - 30.0) < 1e-9


def test_small_ensemble_members():
    e = W.globular_ensemble(s=4, lo=50, hi=200)
    assert e.offsets[0] == 0 and e.offsets[-1] == e.coords.shape[0]
    for s in range(4):
        mem = e.member(s)
        assert mem.n == e.sizes[s]
        assert _min_dist(mem.coords.astype(np.float64)) >= 1.0 - 1e-5


def test_deterministic():
    a = W.ellipsoid_1k()
    b = W.ellipsoid_1k()
    assert np.array_equal(a.coords, b.coords) and np.array_equal(a.types, b.types)
    assert np.array_equal(a.table, b.table)
    r1 = W.random_molecule(5, 10, 4)
    r2 = W.random_molecule(5, 10, 4)
    assert np.array_equal(r1.coords, r2.coords)


def test_non_uniform_grids():
    g = W.log_grid(1e-3, 1.0, 150)
    assert g[0] == pytest.approx(1e-3) and g[-1] == pytest.approx(1.0) and np.all(np.diff(g) > 0)
    r = W.random_grid(5, 0.0, 1.0, 250)
    assert r.dtype == np.float64 and len(r) == 250 and np.all(np.diff(r) > 0) and 0.0 <= r[0] and r[-1] <= 1.0
    assert np.array_equal(r, W.random_grid(5, 0.0, 1.0, 250))
    t = W.two_segment_grid(0.0, 0.1, 1.0, 40, 30)
    assert len(t) == 70 and np.all(np.diff(t) > 0) and t[40] == 0.1 and t[-1] == 1.0
    m = W.random_molecule(3, 10, 0, q=t)
    assert m.table.shape == (5, 70) and np.array_equal(m.q, t)


def test_per_atom_factors():
    m = W.random_molecule(7, 50, 12, q0=0.0, q1=0.6)
    p = W.with_per_atom_factors(m, 3)
    assert p.table.shape == (50, 12) and p.types.dtype == np.int32
    assert sorted(p.types.tolist()) == list(range(50))
    # atom i's row is its element row scaled by 1 + 0.1 (a + b q/qmax), |.| <= 0.2
    ratio = p.table[p.types].astype(np.float64) / m.table[m.types].astype(np.float64)
    assert np.all(np.abs(ratio - 1.0) <= 0.2 + 1e-6)
    assert np.array_equal(p.coords, m.coords)
