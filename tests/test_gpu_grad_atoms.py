"""GPU parity of the coordinate gradient with per-atom form factors (the
per-atom adjoint: many table rows, U_m = w_m f_i(q_m) f_j(q_m) per pair)
against the FP64 oracle.

Bar: the relative norm error and the worst atom's error (tests/gradcheck.py)
within the gradient gate, and the exact identities of Eq. 2's gradient (translation and rotation
invariance) to rounding.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gradcheck import GTOL, assert_grad_close

pytestmark = pytest.mark.gpu


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


def gpu_grad(sd, m, w, ctx=None, with_profile=False):
    import torch

    c = torch.from_numpy(m.coords).cuda()
    t = torch.from_numpy(m.types).cuda()
    tab = torch.from_numpy(m.table).cuda()
    out = sd.debye_grad(c, t, tab, m.q, torch.from_numpy(np.asarray(w, dtype=np.float64)).cuda(),
                        with_profile=with_profile, ctx=ctx)
    if with_profile:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy()


def per_atom_ctx(sd):
    ctx = sd.Context(0)
    ctx.set_form("per_atom")
    return ctx


def check(sd, m, w, ctx=None, atoms=None):
    g = gpu_grad(sd, m, w, ctx=ctx)
    ref = oracle.grad(m.coords, m.types, m.table, m.q, w, atoms=atoms)
    got = g if atoms is None else g[atoms]
    assert_grad_close(got, ref, GTOL, f"per-atom N={m.n} Nq={len(m.q)}")
    return g


@pytest.mark.parametrize("n", [2, 3, 63, 64, 65, 129, 700])
def test_sizes(sd, n):
    say(f"per-atom gradient, T = N = {n}")
    m = W.with_per_atom_factors(W.random_molecule(2100 + n, n, 30, q0=0.0, q1=0.9, extent=3.0 * n ** (1 / 3) + 2.0),
                                2200 + n)
    check(sd, m, np.random.default_rng(n).normal(size=len(m.q)), ctx=per_atom_ctx(sd))


@pytest.mark.parametrize("nq", [1, 2, 64, 65, 250])
def test_q_chunks(sd, nq):
    """Chunks of 64 q values: one, one plus a single value, four."""
    say(f"per-atom gradient, Nq={nq}")
    q0 = 0.3 if nq == 1 else 0.0  # (a single q = 0 has a zero gradient)
    m = W.with_per_atom_factors(W.random_molecule(2120 + nq, 500, nq, q0=q0, q1=0.8, extent=20.0), 2130 + nq)
    check(sd, m, np.random.default_rng(nq).normal(size=nq), ctx=per_atom_ctx(sd))


def test_grid_without_zero_and_log_grid(sd):
    say("per-atom gradient, grid without q = 0 and a log grid (direct variant)")
    m = W.with_per_atom_factors(W.random_molecule(2140, 600, 70, q0=0.05, q1=0.7, extent=22.0), 2141)
    check(sd, m, np.random.default_rng(1).normal(size=len(m.q)), ctx=per_atom_ctx(sd))
    m = W.with_per_atom_factors(W.random_molecule(2142, 600, 0, q=W.log_grid(1e-3, 1.0, 90), extent=22.0), 2143)
    check(sd, m, np.random.default_rng(2).normal(size=len(m.q)), ctx=per_atom_ctx(sd))


def test_forced_form_matches_type_form(sd):
    say("gradient T=5: per-atom form forced vs the type form")
    m = W.random_molecule(2150, 1200, 60, t=5, q0=0.0, q1=1.0, extent=30.0, widths=[0.3, 0.6, 0.9, 1.2, 1.5])
    w = np.random.default_rng(3).normal(size=len(m.q))
    g_pa, I_pa = gpu_grad(sd, m, w, ctx=per_atom_ctx(sd), with_profile=True)
    g_ty, I_ty = gpu_grad(sd, m, w, with_profile=True)
    ref = oracle.grad(m.coords, m.types, m.table, m.q, w)
    for g, what in ((g_pa, "per-atom form"), (g_ty, "type form")):
        assert_grad_close(g, ref, GTOL, what)
    Iref = oracle.profile(m.coords, m.types, m.table, m.q)
    for I in (I_pa, I_ty):
        assert np.max(np.abs(I - Iref) / Iref) <= 1e-6


def test_identities(sd):
    """sum_i g_i = 0 and sum_i x_i x g_i = 0 (Eq. 2 depends on distances
    only), relative to the size of the terms."""
    say("per-atom gradient: translation and rotation identities, T = N = 3000")
    m = W.with_per_atom_factors(W.random_molecule(2160, 3000, 80, q0=0.0, q1=1.0, extent=40.0), 2161)
    g = gpu_grad(sd, m, np.random.default_rng(4).normal(size=len(m.q)), ctx=per_atom_ctx(sd))
    x = m.coords.astype(np.float64)
    scale = np.abs(g).sum()
    assert np.abs(g.sum(axis=0)).max() <= 1e-6 * scale
    torque = np.cross(x - x.mean(axis=0), g).sum(axis=0)
    assert np.abs(torque).max() <= 1e-6 * scale * np.abs(x - x.mean(axis=0)).max()


def test_autograd_many_rows(sd):
    """Autograd through DebyeProfile with 5,000 table rows: coordinate and
    table gradients together, sampled against the oracle."""
    import torch

    say("autograd with T = N = 5000: coordinates and table")
    m = W.with_per_atom_factors(W.random_molecule(2170, 5000, 40, q0=0.0, q1=0.6, extent=42.0), 2171)
    x = torch.from_numpy(m.coords).cuda().requires_grad_(True)
    f = torch.from_numpy(m.table).cuda().requires_grad_(True)
    t = torch.from_numpy(m.types).cuda()
    I = sd.DebyeProfile.apply(x, t, f, m.q)
    w = np.random.default_rng(6).normal(size=len(m.q))
    (I * torch.from_numpy(w).cuda()).sum().backward()
    sub = np.arange(0, 5000, 97)
    ref_c = oracle.grad(m.coords, m.types, m.table, m.q, w, atoms=sub)
    gc = x.grad.double().cpu().numpy()[sub]
    assert_grad_close(gc, ref_c, GTOL, "autograd, 5,000 rows")
    rows = m.types[sub]
    ref_t = oracle.grad_table(m.coords, m.types, m.table, m.q, w)[rows]
    gt = f.grad.double().cpu().numpy()[rows]
    assert np.linalg.norm(gt - ref_t) / np.linalg.norm(ref_t) <= GTOL
