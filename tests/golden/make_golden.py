"""Writes the stored oracle profiles used by the full-size parity tests.

Every value written here comes from the FP64 CPU oracle (``oracle/``) applied
to the seeded workloads of ``workloads.py``; nothing is taken from the HIP
library.  Run from the repository root:

    python tests/golden/make_golden.py [name ...]

Each output file ``<name>.txt`` holds one line per q point:
``q_m  I(q_m)  A(q_m)`` with A = sum |f f sinc| (kappa = A / I); the
ensemble file prefixes each line with the structure's index.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def profile_target(name: str):
    if name == "lattice_20k_target":
        m = workloads.lattice_20k()
        return m.extra["target_coords"], m.types, m.table, m.q
    m = workloads.WORKLOADS[name]()
    return m.coords, m.types, m.table, m.q


def write(name: str) -> None:
    coords, types, table, q = profile_target(name)
    t0 = time.time()
    I, A = oracle.profile(coords, types, table, q, with_abs=True)
    dt = time.time() - t0
    path = os.path.join(HERE, f"{name}.txt")
    with open(path, "w") as fh:
        fh.write(f"# FP64 oracle profile of workload {name}: N={len(types)} Nq={len(q)} "
                 f"({dt:.1f} s on {oracle.max_threads()} threads)\n")
        fh.write("# q  I(q)  A(q)=sum|f f sinc|\n")
        for qm, Im, Am in zip(q, I, A):
            fh.write(f"{float(qm)!r} {float(Im)!r} {float(Am)!r}\n")
    print(f"{name}: {dt:.1f} s -> {path}", flush=True)


# Members of the 256-structure ensemble (globular, 500..8,000 atoms) whose
# profiles are stored: the largest, the smallest, and six drawn with a fixed
# seed from the rest.
ENSEMBLE_FILE = "globular_ensemble_members"


def ensemble_members(sizes) -> list[int]:
    sizes = np.asarray(sizes)
    big, small = int(np.argmax(sizes)), int(np.argmin(sizes))
    rest = [k for k in range(len(sizes)) if k not in (big, small)]
    pick = np.random.default_rng(20260).choice(rest, size=6, replace=False)
    return [big, small] + sorted(int(k) for k in pick)


def write_ensemble() -> None:
    e = workloads.globular_ensemble()
    members = ensemble_members(e.sizes)
    path = os.path.join(HERE, f"{ENSEMBLE_FILE}.txt")
    t0 = time.time()
    rows = []
    for s in members:
        m = e.member(s)
        I, A = oracle.profile(m.coords, m.types, m.table, m.q, with_abs=True)
        rows += [(s, qm, Im, Am) for qm, Im, Am in zip(m.q, I, A)]
    dt = time.time() - t0
    with open(path, "w") as fh:
        fh.write(f"# FP64 oracle profiles of members {members} of globular_ensemble (sizes "
                 f"{[int(e.sizes[s]) for s in members]}, Nq={len(e.q)}) ({dt:.1f} s on {oracle.max_threads()} threads)\n")
        fh.write("# structure  q  I(q)  A(q)=sum|f f sinc|\n")
        for s, qm, Im, Am in rows:
            fh.write(f"{s} {float(qm)!r} {float(Im)!r} {float(Am)!r}\n")
    print(f"{ENSEMBLE_FILE}: {dt:.1f} s -> {path}", flush=True)


def load_ensemble():
    """{structure: (q, I, A)} from the stored ensemble members."""
    data = np.loadtxt(os.path.join(HERE, f"{ENSEMBLE_FILE}.txt"), dtype=np.float64)
    out = {}
    for s in np.unique(data[:, 0]).astype(int):
        d = data[data[:, 0] == s]
        out[int(s)] = (d[:, 1], d[:, 2], d[:, 3])
    return out


# The differentiation workload's chi^2 gradient at sampled atoms: weights
# w_m = dchi2/dI_m from the oracle profile of the lattice and its stored
# target, the oracle gradient at 48 random atoms plus block and strip edges.
GRAD_FILE = "lattice_20k_grad"
GRAD_ATOMS_EDGES = (0, 1, 63, 64, 127, 128, 129, 255, 256, 383, 384, 10239, 10240, 19967, 19968, 19998, 19999)


def lattice_grad_atoms(n: int) -> np.ndarray:
    rnd = np.random.default_rng(4).choice(n, size=48, replace=False)
    return np.unique(np.concatenate([rnd, np.array(GRAD_ATOMS_EDGES)]))


def write_lattice_grad() -> None:
    m = workloads.lattice_20k()
    _, I, _ = load("lattice_20k")
    _, target, _ = load("lattice_20k_target")
    _, w = oracle.chi2(I, target)
    atoms = lattice_grad_atoms(m.n)
    t0 = time.time()
    g = oracle.grad(m.coords, m.types, m.table, m.q, w, atoms=atoms)
    dt = time.time() - t0
    path = os.path.join(HERE, f"{GRAD_FILE}.txt")
    with open(path, "w") as fh:
        fh.write(f"# FP64 oracle chi^2 gradient of lattice_20k at {len(atoms)} atoms, weights from the oracle "
                 f"profile lattice_20k.txt and target lattice_20k_target.txt ({dt:.1f} s)\n")
        fh.write("# w_m (one line, Nq values), then: atom gx gy gz\n")
        fh.write(" ".join(f"{float(v)!r}" for v in w) + "\n")
        for a, row in zip(atoms, g):
            fh.write(f"{int(a)} {float(row[0])!r} {float(row[1])!r} {float(row[2])!r}\n")
    print(f"{GRAD_FILE}: {dt:.1f} s -> {path}", flush=True)


def load_lattice_grad():
    """(w [Nq], atoms [k], g [k, 3]) of the stored chi^2 gradient."""
    with open(os.path.join(HERE, f"{GRAD_FILE}.txt")) as fh:
        lines = [ln for ln in fh if not ln.startswith("#")]
    w = np.array([float(v) for v in lines[0].split()])
    rows = np.array([[float(v) for v in ln.split()] for ln in lines[1:]])
    return w, rows[:, 0].astype(np.int64), rows[:, 1:4]


def load(name: str):
    """(q, I, A) arrays from a stored file."""
    data = np.loadtxt(os.path.join(HERE, f"{name}.txt"), dtype=np.float64)
    return data[:, 0], data[:, 1], data[:, 2]


if __name__ == "__main__":
    names = sys.argv[1:] or ["ellipsoid_1k", "globular_10k", "lattice_20k_target", "lattice_20k", "dna_rod_50k",
                             ENSEMBLE_FILE, GRAD_FILE]
    for n in names:
        if n == ENSEMBLE_FILE:
            write_ensemble()
        elif n == GRAD_FILE:
            write_lattice_grad()
        else:
            write(n)
