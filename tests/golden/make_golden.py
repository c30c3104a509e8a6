"""Writes the stored oracle profiles used by the full-size parity tests.

Every value written here comes from the FP64 CPU oracle (``oracle/``) applied
to the seeded workloads of ``workloads.py``; nothing is taken from the HIP
library.  Run from the repository root:

    python tests/golden/make_golden.py [name ...]

Each output file ``<name>.txt`` holds one line per q point:
``q_m  I(q_m)  A(q_m)`` with A = sum |f f sinc| (kappa = A / I).
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


def load(name: str):
    """(q, I, A) arrays from a stored file."""
    data = np.loadtxt(os.path.join(HERE, f"{name}.txt"), dtype=np.float64)
    return data[:, 0], data[:, 1], data[:, 2]


if __name__ == "__main__":
    names = sys.argv[1:] or ["ellipsoid_1k", "globular_10k", "lattice_20k_target", "dna_rod_50k"]
    for n in names:
        write(n)
