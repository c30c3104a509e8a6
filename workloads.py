"""Seeded synthetic molecules for the Debye-summation workloads.

This module only *draws inputs*: atom positions, atom types, the per-type
form-factor table sampled on the q grid, and the q grid itself.  It holds
none of the summation's arithmetic, so both the FP64 CPU oracle and the HIP
library can be fed from it without sharing any code of the method.

The paper times "randomly generated proteins" (Results section, Table 1) of
1k-100k atoms on uniform 50-100 point profiles over 0 < q <= 1 1/Angstrom,
and cites elongated DNA/RNA-like molecules as the case where direct summation
wins (Background, the q^2 D^2 > N argument).  Its generator is not given, so
the recipes below stand in for it; every choice is listed with the workload.

All arrays are returned as numpy arrays with the exact dtypes the library
takes: coords float32 [N,3] (Angstrom), types int32 [N], table float32
[T,Nq], q float64 [Nq] (1/Angstrom).
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 13062258

# Element mix used by the protein-like workloads: H, C, N, O, S.
TYPE_PROBS = (0.45, 0.30, 0.08, 0.10, 0.07)
TYPE_Z = (1.0, 6.0, 7.0, 8.0, 16.0)
TYPE_B = 1.0  # Angstrom^2, Gaussian width of every element's form factor

# Density of the 10,000-atom globular workload: 10,000 atoms in a 30 A sphere.
GLOBULAR_DENSITY = 10000.0 / (4.0 / 3.0 * math.pi * 30.0 ** 3)


@dataclass
class Molecule:
    """One synthetic structure plus its q grid and per-type form-factor table."""

    name: str
    coords: np.ndarray  # float32 [N,3]
    types: np.ndarray  # int32 [N]
    table: np.ndarray  # float32 [T,Nq]
    q: np.ndarray  # float64 [Nq]
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.coords.shape[0])


@dataclass
class Ensemble:
    """S structures concatenated along the atom axis, with host offsets."""

    name: str
    coords: np.ndarray  # float32 [sum N, 3]
    types: np.ndarray  # int32 [sum N]
    offsets: np.ndarray  # int64 [S+1]
    table: np.ndarray  # float32 [T,Nq]
    q: np.ndarray  # float64 [Nq]

    @property
    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    def member(self, s: int) -> Molecule:
        a, b = int(self.offsets[s]), int(self.offsets[s + 1])
        return Molecule(f"{self.name}[{s}]", self.coords[a:b], self.types[a:b], self.table, self.q)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def q_grid(a: float, b: float, nq: int) -> np.ndarray:
    """Uniform grid with both end points, in FP64 (numpy.linspace)."""
    return np.linspace(a, b, nq, dtype=np.float64)


# Non-uniform grids.  Measured SAS curves are often sampled on logarithmic
# grids or on a fine low-q (Guinier) segment followed by a coarse one; these
# exercise the direct evaluation path of the library.

def log_grid(a: float, b: float, nq: int) -> np.ndarray:
    """nq points geometrically spaced on [a, b], a > 0."""
    return np.geomspace(a, b, nq, dtype=np.float64)


def random_grid(seed: int, a: float, b: float, nq: int) -> np.ndarray:
    """nq distinct sorted points drawn uniformly on [a, b]."""
    rng = rng_for(seed)
    while True:
        q = np.sort(rng.uniform(a, b, size=nq))
        if nq < 2 or np.all(np.diff(q) > 0):
            return q.astype(np.float64)


def two_segment_grid(a: float, mid: float, b: float, n1: int, n2: int) -> np.ndarray:
    """n1 uniform points on [a, mid) then n2 uniform points on [mid, b]."""
    return np.concatenate([np.linspace(a, mid, n1, endpoint=False), np.linspace(mid, b, n2)]).astype(np.float64)


def gaussian_table(z, b, q) -> np.ndarray:
    """Rows f_t(q_m) = Z_t exp(-B_t q_m^2), evaluated in FP64 and rounded once to FP32.

    ``b`` is a scalar (every type shares the width) or one width per type; a
    per-type width gives a form-factor product that does not separate into a
    common q-dependence, which tests use to catch a kernel that assumes it.
    """
    z = np.asarray(z, dtype=np.float64)
    b = np.broadcast_to(np.asarray(b, dtype=np.float64), z.shape)
    q = np.asarray(q, dtype=np.float64)
    return (z[:, None] * np.exp(-b[:, None] * q[None, :] ** 2)).astype(np.float32)


def draw_types(rng: np.random.Generator, n: int, probs=TYPE_PROBS) -> np.ndarray:
    return rng.choice(len(probs), size=n, p=np.asarray(probs, dtype=np.float64)).astype(np.int32)


def uniform_ellipsoid(rng: np.random.Generator, n: int, axes) -> np.ndarray:
    """n points uniform inside an ellipsoid, by rejection from its bounding box."""
    ax = np.asarray(axes, dtype=np.float64)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        cand = rng.uniform(-1.0, 1.0, size=(2 * (n - out.shape[0]) + 16, 3))
        keep = cand[(cand ** 2).sum(axis=1) <= 1.0]
        out = np.vstack([out, keep])
    return out[:n] * ax


def uniform_ball_min_sep(rng: np.random.Generator, n: int, radius: float, min_sep: float) -> np.ndarray:
    """Random sequential addition: uniform candidates in a ball, each kept only if
    it lies at least ``min_sep`` from every atom kept before it.  A cell grid of
    edge ``min_sep`` makes each test look at the 27 surrounding cells only."""
    cell = float(min_sep)
    grid: dict[tuple[int, int, int], list[int]] = {}
    pts = np.empty((n, 3), dtype=np.float64)
    count = 0
    sep2 = min_sep * min_sep
    batch = 4096
    while count < n:
        cand = rng.uniform(-radius, radius, size=(batch, 3))
        cand = cand[(cand ** 2).sum(axis=1) <= radius * radius]
        for p in cand:
            cx, cy, cz = (int(math.floor(p[0] / cell)), int(math.floor(p[1] / cell)), int(math.floor(p[2] / cell)))
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        lst = grid.get((cx + dx, cy + dy, cz + dz))
                        if lst is None:
                            continue
                        for k in lst:
                            d = pts[k] - p
                            if d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < sep2:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                pts[count] = p
                grid.setdefault((cx, cy, cz), []).append(count)
                count += 1
                if count == n:
                    break
    return pts


def double_helix_rod(rng: np.random.Generator, n: int) -> np.ndarray:
    """DNA-like rod: two helical strands (radius 10 A, pitch 34 A, 20 atoms per
    3.4 A rise per strand, Gaussian jitter of 1.5 A per coordinate) holding 80%
    of the atoms, the rest uniform in a 4 A-radius core cylinder of the same
    length; centred on the origin."""
    per_rise = 40  # 20 atoms per strand, two strands
    n_rise = int(round(0.8 * n / per_rise))
    n_strand = n_rise * per_rise
    n_core = n - n_strand
    length = n_rise * 3.4
    k = np.arange(n_rise * 20, dtype=np.float64)
    z = (k // 20 + (k % 20) / 20.0) * 3.4
    strands = []
    for s in (0, 1):
        phi = 2.0 * math.pi * z / 34.0 + s * math.pi
        strands.append(np.stack([10.0 * np.cos(phi), 10.0 * np.sin(phi), z], axis=1))
    helix = np.concatenate(strands, axis=0)
    helix += rng.normal(0.0, 1.5, size=helix.shape)
    rr = 4.0 * np.sqrt(rng.uniform(0.0, 1.0, size=n_core))
    th = rng.uniform(0.0, 2.0 * math.pi, size=n_core)
    zc = rng.uniform(0.0, length, size=n_core)
    core = np.stack([rr * np.cos(th), rr * np.sin(th), zc], axis=1)
    pts = np.concatenate([helix, core], axis=0)
    pts[:, 2] -= length / 2.0
    return pts


def jittered_lattice(rng: np.random.Generator, n: int, shape=(19, 19, 57), spacing=4.0, jitter=0.4) -> np.ndarray:
    """n sites chosen by seeded permutation from a cubic lattice, each moved by
    U(-jitter, jitter) per coordinate; centred on the origin."""
    gx, gy, gz = np.meshgrid(*(np.arange(s, dtype=np.float64) for s in shape), indexing="ij")
    sites = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1) * spacing
    if n > sites.shape[0]:
        raise ValueError("lattice too small")
    pick = rng.permutation(sites.shape[0])[:n]
    pts = sites[np.sort(pick)]
    pts += rng.uniform(-jitter, jitter, size=pts.shape)
    pts -= (np.asarray(shape, dtype=np.float64) - 1.0) * spacing / 2.0
    return pts


def _finish(name, pts, types, table, q, **extra) -> Molecule:
    return Molecule(name, np.ascontiguousarray(pts, dtype=np.float32), np.ascontiguousarray(types, dtype=np.int32),
                    np.ascontiguousarray(table, dtype=np.float32), np.ascontiguousarray(q, dtype=np.float64), extra)


# ----------------------------------------------------------------------------
# The five workloads (index = the seed offset)
# ----------------------------------------------------------------------------

def ellipsoid_1k(n: int = 1000, nq: int = 64, seed: int = BASE_SEED + 0) -> Molecule:
    """1,000 atoms uniform in an ellipsoid (15/12/10 A), 5 element types,
    64 q on [0, 0.5]."""
    rng = rng_for(seed)
    pts = uniform_ellipsoid(rng, n, (15.0, 12.0, 10.0))
    types = draw_types(rng, n)
    q = q_grid(0.0, 0.5, nq)
    return _finish("ellipsoid_1k", pts, types, gaussian_table(TYPE_Z, TYPE_B, q), q)


def globular_10k(n: int = 10000, nq: int = 100, seed: int = BASE_SEED + 1, radius: float = 30.0) -> Molecule:
    """10,000 atoms uniform in a 30 A sphere with a 1 A minimum separation,
    5 element types, 100 q on [0, 1]."""
    rng = rng_for(seed)
    pts = uniform_ball_min_sep(rng, n, radius, 1.0)
    types = draw_types(rng, n)
    q = q_grid(0.0, 1.0, nq)
    return _finish("globular_10k", pts, types, gaussian_table(TYPE_Z, TYPE_B, q), q)


@functools.lru_cache(maxsize=4)
def _rod(n: int, seed: int):
    rng = rng_for(seed)
    pts = double_helix_rod(rng, n)
    types = draw_types(rng, n)
    return pts, types


def dna_rod_50k(n: int = 50000, nq: int = 200, seed: int = BASE_SEED + 2, q=None) -> Molecule:
    """50,000-atom double-helix rod (about 3,400 A long), 5 element types,
    200 q on [0, 1]."""
    pts, types = _rod(n, seed)
    q = q_grid(0.0, 1.0, nq) if q is None else np.asarray(q, dtype=np.float64)
    return _finish("dna_rod_50k", pts.copy(), types.copy(), gaussian_table(TYPE_Z, TYPE_B, q), q)


def globular(n: int, nq: int = 200, q1: float = 1.0, seed: int = BASE_SEED + 70) -> Molecule:
    """n atoms in a sphere at the 10,000-atom workload's density (1 A minimum
    separation), the 5-type mix, nq q on [0, q1]: a large compact molecule,
    the case where orientation averaging pays at low q."""
    rng = rng_for(seed)
    pts = uniform_ball_min_sep(rng, n, globular_radius(n), 1.0)
    types = draw_types(rng, n)
    q = q_grid(0.0, q1, nq)
    return _finish(f"globular_{n}", pts, types, gaussian_table(TYPE_Z, TYPE_B, q), q)


def globular_radius(n: int) -> float:
    """Radius that keeps the 10,000-atom workload's density for n atoms."""
    return (3.0 * n / (4.0 * math.pi * GLOBULAR_DENSITY)) ** (1.0 / 3.0)


def ensemble_sizes(s: int = 256, lo: int = 500, hi: int = 8000, seed: int = BASE_SEED + 3) -> np.ndarray:
    rng = rng_for(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=s))).astype(np.int64)


def globular_ensemble(s: int = 256, nq: int = 100, lo: int = 500, hi: int = 8000, seed: int = BASE_SEED + 3) -> Ensemble:
    """s globular structures with log-uniform atom counts in [lo, hi], each drawn
    at the 10,000-atom workload's density with seed BASE_SEED+1000+index,
    sharing one 100-point grid on [0, 0.8]."""
    sizes = ensemble_sizes(s, lo, hi, seed)
    coords, types = [], []
    for k, n in enumerate(sizes):
        rng = rng_for(BASE_SEED + 1000 + k)
        coords.append(uniform_ball_min_sep(rng, int(n), globular_radius(int(n)), 1.0))
        types.append(draw_types(rng, int(n)))
    offsets = np.zeros(s + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    q = q_grid(0.0, 0.8, nq)
    return Ensemble("globular_ensemble", np.ascontiguousarray(np.concatenate(coords), dtype=np.float32),
                    np.ascontiguousarray(np.concatenate(types), dtype=np.int32), offsets,
                    gaussian_table(TYPE_Z, TYPE_B, q), q)


def lattice_20k(n: int = 20000, nq: int = 100, seed: int = BASE_SEED + 4, perturb: float = 0.5) -> Molecule:
    """20,000 coarse-grained pseudo-atoms on a jittered 4 A cubic lattice
    (19x19x57 sites, 1:1:3 box), one type f(q) = 10 exp(-2 q^2), 100 q on
    [0, 0.5].  ``extra['target_coords']`` is a copy moved by N(0, perturb^2)
    per coordinate (seed+1); the fit target profile is computed from it."""
    rng = rng_for(seed)
    pts = jittered_lattice(rng, n)
    types = np.zeros(n, dtype=np.int32)
    q = q_grid(0.0, 0.5, nq)
    table = gaussian_table((10.0,), 2.0, q)
    rng2 = rng_for(seed + 1)
    tgt = pts + rng2.normal(0.0, perturb, size=pts.shape)
    return _finish("lattice_20k", pts, types, table, q, target_coords=np.ascontiguousarray(tgt, dtype=np.float32))


def with_per_atom_factors(m: Molecule, seed: int, spread: float = 0.1, shuffle: bool = True) -> Molecule:
    """The same atoms with one table row per atom (T = N): atom i's element
    factor scaled by 1 + spread (a_i + b_i q / q_max), a_i, b_i ~ U(-1, 1), the
    kind of per-atom correction a hydration or excluded-volume model applies.
    With ``shuffle`` the row of atom i is a random permutation index, so that
    atom order and row order differ."""
    rng = rng_for(seed)
    n = m.n
    a = rng.uniform(-1.0, 1.0, size=n)
    b = rng.uniform(-1.0, 1.0, size=n)
    qmax = max(float(np.max(m.q)), 1e-30) if len(m.q) else 1.0
    rows = rng.permutation(n).astype(np.int32) if shuffle else np.arange(n, dtype=np.int32)
    scale = 1.0 + spread * (a[:, None] + b[:, None] * (m.q[None, :] / qmax))
    per_atom = m.table.astype(np.float64)[m.types] * scale  # row i belongs to atom i
    table = np.empty_like(per_atom)
    table[rows] = per_atom
    return Molecule(m.name + "_per_atom", m.coords, rows, np.ascontiguousarray(table, dtype=np.float32), m.q,
                    dict(m.extra))


def with_random_rows(m: Molecule, t: int, seed: int) -> Molecule:
    """The same atoms with t table rows Z_r exp(-B_r q^2), Z_r ~ U(1, 16) and
    B_r ~ U(0.2, 1.5) (not separable), each atom's row drawn uniformly: with t
    comparable to the atom count some rows are shared and some unused."""
    rng = rng_for(seed)
    rows = rng.integers(0, t, size=m.n).astype(np.int32)
    z = rng.uniform(1.0, 16.0, size=t)
    b = rng.uniform(0.2, 1.5, size=t)
    table = (z[:, None] * np.exp(-b[:, None] * m.q[None, :] ** 2)).astype(np.float32)
    return Molecule(m.name + f"_rows{t}", m.coords, rows, table, m.q, dict(m.extra))


WORKLOADS = {
    "ellipsoid_1k": ellipsoid_1k,
    "globular_10k": globular_10k,
    "dna_rod_50k": dna_rod_50k,
    "lattice_20k": lattice_20k,
}


def random_molecule(seed: int, n: int, nq: int, t: int = 5, q0: float = 0.0, q1: float = 0.5, extent: float = 20.0,
                    widths=None, q=None) -> Molecule:
    """Small generic case for edge tests: n atoms uniform in a cube of edge
    ``extent``, t types drawn uniformly, a table with Z_t = 1 + t and a
    per-type Gaussian width (non-separable by default).  ``q`` replaces the
    uniform grid (q0, q1, nq) when given."""
    rng = rng_for(seed)
    pts = rng.uniform(-extent / 2, extent / 2, size=(n, 3))
    types = rng.integers(0, t, size=n).astype(np.int32)
    q = q_grid(q0, q1, nq) if q is None else np.asarray(q, dtype=np.float64)
    z = 1.0 + np.arange(t, dtype=np.float64)
    if widths is None:
        widths = 0.5 + 0.25 * np.arange(t, dtype=np.float64)
    return _finish(f"random_{seed}", pts, types, gaussian_table(z, widths, q), q)
