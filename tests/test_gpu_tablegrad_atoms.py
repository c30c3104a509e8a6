"""GPU parity of the table gradient in its per-atom form (many table rows:
per-atom form factors, T up to N and beyond 64) against the FP64 oracle.

The form sums, for every atom, S_i(q) = sum_j f_j(q) sinc(q r_ij) over the
whole square of pairs and adds S_i by type (dI/df_t = 2 sum over atoms of type
t of S_i).  Bar: per type row, ||g_gpu - g_oracle|| / ||g_oracle|| <= 1e-5
(the gradient gate); rows of types no atom holds are exactly zero; the
profile returned beside it within 1e-6 per q.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

GTOL = 1e-5


@pytest.fixture(scope="module")
def sd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_2258_amd as mod

    return mod


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def per_atom(m, seed, t=None):
    """m with one table row per atom (t = None) or t rows shared at random."""
    return W.with_per_atom_factors(m, seed) if t is None else W.with_random_rows(m, t, seed)


def run(sd, m, w, ctx=None, with_profile=True):
    import torch

    c = torch.from_numpy(m.coords).cuda()
    t = torch.from_numpy(m.types).cuda()
    tab = torch.from_numpy(m.table).cuda()
    out = sd.debye_grad_table(c, t, tab, m.q, torch.from_numpy(np.asarray(w, dtype=np.float64)).cuda(),
                              with_profile=with_profile, ctx=ctx)
    if with_profile:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy(), None


def check(sd, m, w, pick=None, ctx=None):
    g, I = run(sd, m, w, ctx=ctx)
    assert np.all(np.isfinite(g))
    qi = np.arange(len(m.q)) if pick is None else pick
    ref = oracle.grad_table(m.coords, m.types, m.table[:, qi], m.q[qi], np.asarray(w)[qi])
    got = g[:, qi]
    present = np.bincount(m.types, minlength=m.table.shape[0]) > 0
    assert np.all(got[~present] == 0.0)
    nz = present & (np.linalg.norm(ref, axis=1) > 0)
    err = np.linalg.norm(got[nz] - ref[nz], axis=1) / np.linalg.norm(ref[nz], axis=1)
    print(f"per-atom table grad: max row rel err {err.max():.3e} over {nz.sum()} rows")
    assert err.max() <= GTOL
    Iref = oracle.profile(m.coords, m.types, m.table[:, qi], m.q[qi])
    assert np.max(np.abs(I[qi] - Iref) / np.abs(Iref)) <= 1e-6
    return g, I


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 129, 700])
def test_one_row_per_atom_sizes(sd, n):
    say(f"per-atom table gradient, T = N = {n}")
    m = per_atom(W.random_molecule(2000 + n, n, 30, t=3, q0=0.0, q1=1.0, extent=3.0 * n ** (1 / 3) + 2.0), n)
    check(sd, m, np.random.default_rng(n).normal(size=len(m.q)))


def test_shared_rows_and_unused_rows(sd):
    """T = 300 rows for 500 atoms drawn at random: some rows shared by several
    atoms (summed in index order), some held by none (exactly zero)."""
    say("per-atom table gradient, T=300 rows shared at random by 500 atoms")
    m = per_atom(W.random_molecule(2030, 500, 40, t=1, q0=0.0, q1=0.9, extent=18.0), 7, t=300)
    assert np.bincount(m.types, minlength=300).min() == 0 and np.bincount(m.types).max() > 1
    check(sd, m, np.random.default_rng(3).normal(size=len(m.q)))


@pytest.mark.parametrize("nq", [1, 2, 250])
def test_q_counts(sd, nq):
    say(f"per-atom table gradient, Nq={nq}")
    m = per_atom(W.random_molecule(2040 + nq, 300, nq, t=1, q0=0.0, q1=0.8, extent=16.0), nq)
    check(sd, m, np.random.default_rng(nq).normal(size=nq))


def test_grid_without_zero_and_log_grid(sd):
    say("per-atom table gradient on a grid without q = 0 and on a log grid (direct form)")
    m = per_atom(W.random_molecule(2050, 600, 45, t=1, q0=0.02, q1=0.7, extent=20.0), 11)
    check(sd, m, np.random.default_rng(8).normal(size=len(m.q)))
    m = per_atom(W.random_molecule(2051, 600, 0, t=1, q=W.log_grid(1e-3, 1.0, 60), extent=20.0), 12)
    check(sd, m, np.random.default_rng(9).normal(size=len(m.q)))


def test_forced_form_matches_type_form(sd):
    """T = 5: the per-atom form (forced) against the per-type sums of the
    forward pass, and both against the oracle."""
    say("table gradient T=5: per-atom form forced vs type form")
    m = W.random_molecule(2060, 900, 50, t=5, q0=0.0, q1=1.0, extent=26.0, widths=[0.3, 0.6, 0.9, 1.2, 1.5])
    w = np.random.default_rng(10).normal(size=len(m.q))
    ctx = sd.Context(0)
    ctx.set_form("per_atom")
    g_atoms, _ = check(sd, m, w, ctx=ctx)
    g_types, _ = check(sd, m, w)
    rel = np.linalg.norm(g_atoms - g_types, axis=1) / np.linalg.norm(g_types, axis=1)
    assert rel.max() <= 2 * GTOL


def test_deterministic(sd):
    say("per-atom table gradient: two calls give the same bits")
    m = per_atom(W.random_molecule(2070, 800, 64, t=1, q0=0.0, q1=1.0, extent=24.0), 13, t=200)
    w = np.random.default_rng(11).normal(size=len(m.q))
    a, Ia = run(sd, m, w)
    b, Ib = run(sd, m, w)
    assert np.array_equal(a, b) and np.array_equal(Ia, Ib)


def test_euler_identity(sd):
    """Eq. 2 is homogeneous of degree 2 in the form factors:
    sum_t f_t dI/df_t = 2 I, here with T = N = 3000."""
    say("per-atom table gradient: Euler identity, T = N = 3000")
    m = per_atom(W.random_molecule(2080, 3000, 80, t=1, q0=0.0, q1=1.0, extent=40.0), 14)
    g, I = run(sd, m, np.ones(len(m.q)))
    lhs = (m.table.astype(np.float64) * g).sum(axis=0)
    assert np.max(np.abs(lhs - 2.0 * I) / np.abs(2.0 * I)) <= 2e-6


def test_globular_10k_one_row_per_atom_sampled(sd):
    """The 10,000-atom globular workload with one row per atom, at full size:
    three q values of the gradient against the oracle."""
    say("per-atom table gradient globular_10k, T = N, sampled q")
    m = per_atom(W.globular_10k(), 15)
    w = np.random.default_rng(12).normal(size=len(m.q))
    check(sd, m, w, pick=np.array([0, 37, 99]))
