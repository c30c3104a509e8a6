"""GPU parity of the table gradient (dL/dtable) against the FP64 oracle.

sas_debye_grad_table returns w_m dI(q_m)/df_t(q_m) for every type t and q.
Bar: per type row, ||g_gpu - g_oracle|| / ||g_oracle|| <= 1e-5 (the
gradient gate), and the profile it can return within 1e-6 per q.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gradcheck import assert_grad_close

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


def to_dev(m):
    import torch

    return (torch.from_numpy(m.coords).cuda(), torch.from_numpy(m.types).cuda(), torch.from_numpy(m.table).cuda())


def gpu_grad_table(sd, m, w, with_profile=False):
    import torch

    c, t, tab = to_dev(m)
    out = sd.debye_grad_table(c, t, tab, m.q, torch.from_numpy(np.asarray(w, dtype=np.float64)).cuda(),
                              with_profile=with_profile)
    if with_profile:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy()


def check(sd, m, w, pick=None):
    g, I = gpu_grad_table(sd, m, w, with_profile=True)
    assert np.all(np.isfinite(g))
    if pick is None:
        ref = oracle.grad_table(m.coords, m.types, m.table, m.q, w)
        got = g
        Iref = oracle.profile(m.coords, m.types, m.table, m.q)
        Igot = I
    else:
        ref = oracle.grad_table(m.coords, m.types, m.table[:, pick], m.q[pick], np.asarray(w)[pick])
        got = g[:, pick]
        Iref = oracle.profile(m.coords, m.types, m.table[:, pick], m.q[pick])
        Igot = I[pick]
    present = np.linalg.norm(ref, axis=1) > 0
    assert np.all(got[~present] == 0.0)
    err = np.linalg.norm(got[present] - ref[present], axis=1) / np.linalg.norm(ref[present], axis=1)
    print(f"table grad: max row rel err {err.max():.3e}")
    assert err.max() <= GTOL
    assert np.max(np.abs(Igot - Iref) / np.abs(Iref)) <= 1e-6
    return g, I


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 300, 1000])
def test_table_grad_sizes(sd, n):
    say(f"table gradient N={n}, T=3")
    m = W.random_molecule(1300 + n, n, 29, t=3, q0=0.0, q1=1.0, extent=3.0 * max(n, 1) ** (1 / 3) + 2.0,
                          widths=[0.4, 0.9, 1.5])
    check(sd, m, np.random.default_rng(n).normal(size=len(m.q)))


@pytest.mark.parametrize("t", [1, 5, 17, 64])
def test_table_grad_type_counts(sd, t):
    """Many types make many I blocks straddle a type boundary (the per-type
    passes over such blocks)."""
    say(f"table gradient T={t}, N=700")
    m = W.random_molecule(1320 + t, 700, 33, t=t, q0=0.0, q1=1.2, extent=22.0, widths=np.linspace(0.2, 1.5, t))
    check(sd, m, np.random.default_rng(t).normal(size=len(m.q)))


@pytest.mark.parametrize("nq", [1, 2, 250])
def test_table_grad_q_counts(sd, nq):
    say(f"table gradient Nq={nq}")
    m = W.random_molecule(1340 + nq, 400, nq, t=4, q0=0.0, q1=0.9, extent=20.0)
    check(sd, m, np.random.default_rng(nq).normal(size=nq))


def test_table_grad_nonuniform_grid(sd):
    say("table gradient on a log grid (direct form)")
    m = W.random_molecule(1350, 800, 0, t=5, q=W.log_grid(1e-3, 1.0, 70), extent=26.0)
    check(sd, m, np.random.default_rng(1).normal(size=len(m.q)))


def test_table_grad_euler_identity(sd):
    """Eq. 2 is homogeneous of degree 2 in the table: sum_t f_t dI/df_t = 2 I."""
    say("table gradient: Euler identity against the returned profile")
    m = W.random_molecule(1360, 1500, 60, t=5, q0=0.0, q1=1.0, extent=30.0)
    g, I = gpu_grad_table(sd, m, np.ones(len(m.q)), with_profile=True)
    lhs = (m.table.astype(np.float64) * g).sum(axis=0)
    assert np.max(np.abs(lhs - 2.0 * I) / np.abs(2.0 * I)) <= 2e-6


def test_table_grad_coincident_atoms(sd):
    say("table gradient with coincident atoms")
    m = W.random_molecule(1370, 300, 25, t=3, q0=0.0, q1=1.0, extent=12.0)
    m.coords[11] = m.coords[2]
    m.coords[299] = m.coords[0]
    check(sd, m, np.random.default_rng(2).normal(size=len(m.q)))


def test_table_grad_many_types(sd):
    """T = 65 is past the per-type sums of the forward pass: the per-atom
    form takes over, same results."""
    say("table gradient T=65 (per-atom form)")
    m = W.random_molecule(1380, 400, 20, t=65, q0=0.0, q1=0.5, extent=14.0, widths=np.linspace(0.2, 1.5, 65))
    check(sd, m, np.random.default_rng(6).normal(size=len(m.q)))


def test_table_grad_autograd(sd):
    import torch

    say("autograd: gradients for coords and table together")
    m = W.random_molecule(1390, 250, 20, t=3, q0=0.0, q1=0.8, extent=14.0)
    c, t, tab = to_dev(m)
    x = c.clone().requires_grad_(True)
    f = tab.clone().requires_grad_(True)
    I = sd.DebyeProfile.apply(x, t, f, m.q)
    w = np.random.default_rng(4).normal(size=len(m.q))
    (I * torch.from_numpy(w).cuda()).sum().backward()
    ref_t = oracle.grad_table(m.coords, m.types, m.table, m.q, w)
    ref_c = oracle.grad(m.coords, m.types, m.table, m.q, w)
    assert f.grad.dtype == torch.float32 and x.grad.dtype == torch.float32
    gt = f.grad.double().cpu().numpy()
    assert np.linalg.norm(gt - ref_t) / np.linalg.norm(ref_t) <= GTOL
    gc = x.grad.double().cpu().numpy()
    assert_grad_close(gc, ref_c, GTOL, "autograd with the table")


def test_table_grad_globular_10k_sampled(sd):
    """The 10,000-atom globular workload at full size: three q values of the
    table gradient against the oracle."""
    say("table gradient globular_10k, sampled q")
    m = W.globular_10k()
    w = np.random.default_rng(5).normal(size=len(m.q))
    check(sd, m, w, pick=np.array([1, 40, 99]))
