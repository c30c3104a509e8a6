"""GPU parity of the forward profile (plain and batched) against the FP64 oracle.

Bar: max over q of |I_gpu - I_oracle| / I_oracle <= 1e-6 (the target stated
for this path), on seeded synthetic molecules.  Every case prints its name
before touching the GPU.
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-6


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


def gpu_profile(sd, m, ctx=None):
    c, t, tab = to_dev(m)
    return sd.debye_profile(c, t, tab, m.q, ctx=ctx).cpu().numpy()


def rel_err(a, b):
    return np.abs(a - b) / np.abs(b)


def check_against_oracle(sd, m, tol=TOL, ctx=None):
    got = gpu_profile(sd, m, ctx=ctx)
    ref = oracle.profile(m.coords, m.types, m.table, m.q)
    err = rel_err(got, ref)
    assert np.all(np.isfinite(got))
    assert err.max() <= tol, f"{m.name}: max rel err {err.max():.3e} at q[{err.argmax()}]"
    return err.max()


def test_ellipsoid_1k(sd):
    say("ellipsoid_1k N=1000 Nq=64")
    e = check_against_oracle(sd, W.ellipsoid_1k())
    print(f"max rel err {e:.3e}")


@pytest.mark.parametrize("n", [0, 1, 2, 3, 63, 64, 65, 127, 255, 256, 257, 513, 1000])
def test_edge_sizes(sd, n):
    say(f"edge size N={n}")
    m = W.random_molecule(100 + n, n, 17, q0=0.0, q1=0.9, extent=3.0 * max(n, 1) ** (1 / 3) + 2.0)
    if n == 0:
        import torch

        out = sd.debye_profile(torch.zeros((0, 3), dtype=torch.float32, device="cuda"),
                               torch.zeros(0, dtype=torch.int32, device="cuda"),
                               torch.from_numpy(m.table).cuda(), m.q).cpu().numpy()
        assert np.all(out == 0.0)
        return
    check_against_oracle(sd, m)


@pytest.mark.parametrize("nq", [1, 2, 7, 16, 50, 64, 99, 100, 101, 200, 257, 450])
def test_q_counts(sd, nq):
    say(f"q count Nq={nq}")
    m = W.random_molecule(300 + nq, 300, nq, q0=0.0, q1=1.0, extent=25.0)
    check_against_oracle(sd, m)


@pytest.mark.parametrize("q0", [0.0, 1e-3, 0.05, 0.37, 2.0])
def test_grid_start(sd, q0):
    say(f"grid start q0={q0}")
    m = W.random_molecule(400, 500, 40, q0=q0, q1=q0 + 0.6, extent=30.0)
    check_against_oracle(sd, m)


def test_paper_grid_50_points(sd):
    # the paper's profiles: 50 uniform points with 0 < q <= 1
    say("paper grid q=m/50, m=1..50")
    m = W.random_molecule(401, 800, 50, q0=0.02, q1=1.0, extent=40.0)
    check_against_oracle(sd, m)


@pytest.mark.parametrize("t", [1, 5, 64, 300])
def test_type_counts_non_separable(sd, t):
    say(f"type count T={t} (per-type widths)")
    m = W.random_molecule(500 + t, 700, 33, t=t, q0=0.0, q1=1.2, extent=22.0,
                          widths=np.linspace(0.2, 1.5, t))
    check_against_oracle(sd, m)


def test_per_atom_form_factors(sd):
    say("T = N per-atom table")
    m = W.random_molecule(601, 150, 20, t=150, q0=0.0, q1=0.8, extent=15.0, widths=np.linspace(0.3, 1.2, 150))
    m.types = np.arange(150, dtype=np.int32)
    check_against_oracle(sd, m)


def test_coincident_atoms(sd):
    say("coincident atoms")
    m = W.random_molecule(602, 200, 25, t=3, q0=0.0, q1=1.0, extent=12.0)
    m.coords[50] = m.coords[10]
    m.coords[51] = m.coords[10]
    m.coords[199] = m.coords[0]
    check_against_oracle(sd, m)


def test_large_q_argument(sd):
    say("long distances and large q (theta up to ~2e4 rad)")
    m = W.random_molecule(603, 400, 30, q0=0.0, q1=5.0, extent=4000.0)
    check_against_oracle(sd, m)


@pytest.mark.parametrize("bj", [64, 128, 256, 512])
@pytest.mark.parametrize("qc", [16, 32, 50, 64, 100, 128, 150, 200])
def test_variants(sd, bj, qc):
    say(f"variant bj={bj} qc={qc}")
    ctx = sd.Context(0)
    ctx.set_variant(bj, qc)
    m = W.random_molecule(700, 1100, 73, q0=0.0, q1=0.7, extent=30.0)
    check_against_oracle(sd, m, ctx=ctx)
    assert ctx.variant() == (bj, qc)


def test_determinism_bitwise(sd):
    say("determinism")
    m = W.random_molecule(800, 3000, 64, q0=0.0, q1=1.0, extent=40.0)
    a = gpu_profile(sd, m)
    b = gpu_profile(sd, m)
    assert np.array_equal(a, b)


def test_invariances(sd):
    say("rotation / translation / permutation invariance")
    m = W.random_molecule(801, 2000, 48, q0=0.0, q1=1.0, extent=35.0)
    base = gpu_profile(sd, m)
    rng = np.random.default_rng(0)
    qm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    m2 = W.Molecule("rot", (m.coords.astype(np.float64) @ qm.T + 5.0).astype(np.float32), m.types, m.table, m.q)
    ref2 = oracle.profile(m2.coords, m2.types, m2.table, m2.q)
    assert rel_err(gpu_profile(sd, m2), ref2).max() <= TOL
    perm = rng.permutation(m.n)
    m3 = W.Molecule("perm", m.coords[perm].copy(), m.types[perm].copy(), m.table, m.q)
    assert rel_err(gpu_profile(sd, m3), base).max() <= 1e-7


def test_power_of_two_scaling_bitwise(sd):
    # r -> 2r and q -> q/2 leave every q*r and every FP32 operation scaled by an
    # exact power of two; the per-pair values y = sin(qr)/r scale by 1/2 exactly.
    say("power-of-two scaling")
    m = W.random_molecule(802, 900, 40, q0=0.0, q1=1.0, extent=30.0)
    a = gpu_profile(sd, m)
    m2 = W.Molecule("x2", (2.0 * m.coords).astype(np.float32), m.types, m.table, m.q / 2.0)
    b = gpu_profile(sd, m2)
    assert np.array_equal(a, b)


def test_globular_10k_vs_stored_oracle(sd):
    from tests.golden.make_golden import load

    say("globular_10k N=10000 Nq=100 (stored oracle profile)")
    m = W.globular_10k()
    q, I, A = load("globular_10k")
    assert np.array_equal(q, m.q)
    got = gpu_profile(sd, m)
    err = rel_err(got, I)
    kappa = A / I
    print(f"max rel err {err.max():.3e} at q[{err.argmax()}] (kappa there {kappa[err.argmax()]:.1f})")
    assert err.max() <= TOL


def test_dna_rod_50k_full_size(sd):
    """The 50,000-atom, 200-q rod at the launch configuration the benchmark
    times: all 200 values against the stored oracle profile if present, and
    six q values against the oracle computed here."""
    say("dna_rod_50k N=50000 Nq=200")
    m = W.dna_rod_50k()
    got = gpu_profile(sd, m)
    pick = np.array([1, 17, 60, 111, 160, 199])
    ref = oracle.profile(m.coords, m.types, m.table[:, pick], m.q[pick])
    err = rel_err(got[pick], ref)
    print("sampled q errors", " ".join(f"{e:.2e}" for e in err))
    assert err.max() <= TOL
    path = os.path.join(os.path.dirname(__file__), "golden", "dna_rod_50k.txt")
    if os.path.exists(path):
        from tests.golden.make_golden import load

        q, I, A = load("dna_rod_50k")
        err = rel_err(got, I)
        print(f"all 200 q: max rel err {err.max():.3e} at q[{err.argmax()}]")
        assert err.max() <= TOL


# ---------------------------------------------------------------------------
# Batched form
# ---------------------------------------------------------------------------

def test_batched_matches_plain_and_oracle(sd):
    import torch

    say("batched: 12 structures of uneven size incl. N=0, N=1")
    sizes = [0, 1, 2, 70, 513, 1000, 64, 257, 3, 1500, 65, 800]
    mols = [W.random_molecule(900 + k, n, 30, q0=0.0, q1=0.8, extent=2.5 * max(n, 1) ** (1 / 3) + 3)
            for k, n in enumerate(sizes)]
    table = mols[0].table
    coords = np.concatenate([mm.coords for mm in mols]).astype(np.float32)
    types = np.concatenate([mm.types for mm in mols]).astype(np.int32)
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    out = sd.debye_profile_batched(torch.from_numpy(coords).cuda(), torch.from_numpy(types).cuda(), off,
                                   torch.from_numpy(table).cuda(), mols[0].q).cpu().numpy()
    # with one tile shape forced for both, a structure's batched result is the
    # plain call's result bit for bit (same tiles, same summation order)
    ctx = sd.Context(0)
    ctx.set_variant(128, 32)
    out_forced = sd.debye_profile_batched(torch.from_numpy(coords).cuda(), torch.from_numpy(types).cuda(), off,
                                          torch.from_numpy(table).cuda(), mols[0].q, ctx=ctx).cpu().numpy()
    for k, mm in enumerate(mols):
        ref = oracle.profile(mm.coords, mm.types, table, mm.q)
        if sizes[k] == 0:
            assert np.all(out[k] == 0.0) and np.all(out_forced[k] == 0.0)
            continue
        assert rel_err(out[k], ref).max() <= TOL, f"structure {k} (N={sizes[k]})"
        assert rel_err(out_forced[k], ref).max() <= TOL, f"structure {k} (N={sizes[k]}), forced variant"
        plain = gpu_profile(sd, W.Molecule("p", mm.coords, mm.types, table, mm.q), ctx=ctx)
        assert np.array_equal(out_forced[k], plain), f"structure {k}"


def test_batched_single_structure_equals_plain(sd):
    import torch

    say("batched S=1")
    m = W.random_molecule(990, 777, 21)
    out = sd.debye_profile_batched(torch.from_numpy(m.coords).cuda(), torch.from_numpy(m.types).cuda(),
                                   [0, m.n], torch.from_numpy(m.table).cuda(), m.q).cpu().numpy()
    assert np.array_equal(out[0], gpu_profile(sd, m))


def test_errors_are_reported(sd):
    import torch

    say("error paths")
    m = W.random_molecule(991, 10, 5)
    c, t, tab = to_dev(m)
    for bad in ([0.0, 0.2, 0.1, 0.4, 0.5], [-0.1, 0.1, 0.2, 0.3, 0.4], [0.0, 0.1, np.nan, 0.3, 0.4],
                [0.0, 0.1, 0.1, 0.3, 0.4]):
        with pytest.raises(sd.SasError) as e:
            sd.debye_profile(c, t, tab, np.array(bad))
        assert e.value.status == 2, bad
    ctx = sd.Context(0)
    n = m.n
    import ctypes

    from paper_1306_2258_amd import _lib

    lib = _lib.load()
    qh = np.ascontiguousarray(m.q)
    out = torch.empty(5, dtype=torch.float64, device="cuda")
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    st = lib.sas_debye_profile(ctx.handle, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(t.data_ptr()), n,
                               ctypes.c_void_p(tab.data_ptr()), 5, qh.ctypes.data_as(ctypes.c_void_p), 5,
                               ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), 256, None)
    assert st == 4  # workspace too small


# ---------------------------------------------------------------------------
# Batched plan: tuned tile shape, captured graph, replays after in-place updates
# ---------------------------------------------------------------------------

def _ensemble(sizes, seed=3000, nq=40):
    mols = [W.random_molecule(seed + k, n, nq, q0=0.0, q1=0.8, extent=2.5 * max(n, 1) ** (1 / 3) + 3)
            for k, n in enumerate(sizes)]
    coords = np.concatenate([mm.coords for mm in mols]).astype(np.float32)
    types = np.concatenate([mm.types for mm in mols]).astype(np.int32)
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return mols, coords, types, off


def test_plan_replays_match_eager_and_oracle(sd):
    import torch

    say("batched plan: tune, capture, replay x3 with in-place coordinate updates")
    sizes = [900, 130, 2, 1, 0, 2100, 640, 65]
    mols, coords, types, off = _ensemble(sizes)
    table, q = mols[0].table, mols[0].q
    ctx = sd.Context(0)
    c = torch.from_numpy(coords).cuda()
    t = torch.from_numpy(types).cuda()
    tab = torch.from_numpy(table).cuda()
    plan = sd.BatchedPlan(c, t, off, tab, q, ctx=ctx)
    rng = np.random.default_rng(11)
    for rep in range(3):
        got = plan.execute().clone()
        torch.cuda.synchronize()
        bj, qc = ctx.variant()
        # eager work between replays: an eager batched call with the same shape
        ctx2 = sd.Context(0)
        ctx2.set_variant(bj, qc)
        eager = sd.debye_profile_batched(c, t, off, tab, q, ctx=ctx2)
        torch.cuda.synchronize()
        assert torch.equal(got, eager), f"replay {rep} differs from the eager call"
        host = c.cpu().numpy()
        for k, n in enumerate(sizes):
            if n == 0:
                assert torch.all(got[k] == 0)
                continue
            ref = oracle.profile(host[off[k]:off[k + 1]], types[off[k]:off[k + 1]], table, q)
            assert rel_err(got[k].cpu().numpy(), ref).max() <= TOL, f"replay {rep} structure {k}"
        # rewrite the coordinates in place: rotate and shift every structure
        qm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        new = (host.astype(np.float64) @ qm.T + rng.normal(size=3)).astype(np.float32)
        new[: off[1]] += rng.normal(scale=0.3, size=(off[1], 3)).astype(np.float32)  # change one structure's shape
        c.copy_(torch.from_numpy(new).cuda())
        torch.cuda.synchronize()
    plan.close()


@pytest.mark.parametrize("nq", [64, 200, 450])
def test_persistent_launch_matches_grid(sd, nq):
    """The persistent launch of the pair kernel (one-wave work-groups pulling
    (strip, q chunk) items from a counter) gives the grid launch's results bit
    for bit: single structures of several sizes (450 q: three chunks, so the
    item decode walks chunks), a batched call with empty and one-atom
    structures, repeated calls (the counter is re-zeroed each call), and the
    launch each call reports."""
    import torch

    say(f"persistent vs grid launch, Nq={nq}")
    grid_ctx, pers_ctx = sd.Context(0), sd.Context(0)
    grid_ctx.set_form("grid")
    pers_ctx.set_form("persistent")
    auto_ctx = sd.Context(0)
    for n in (2, 65, 700, 3000):
        m = W.random_molecule(4000 + n + nq, n, nq, q0=0.0, q1=1.0, extent=3.0 * n ** (1 / 3) + 4)
        a = gpu_profile(sd, m, ctx=grid_ctx)
        assert grid_ctx.launch() == "grid"
        for _ in range(2):
            b = gpu_profile(sd, m, ctx=pers_ctx)
            assert pers_ctx.launch() == "persistent"
            assert np.array_equal(a, b), f"N={n}"
        c = gpu_profile(sd, m, ctx=auto_ctx)
        assert auto_ctx.launch() == "persistent" and np.array_equal(a, c)
    ref = oracle.profile(m.coords, m.types, m.table, m.q)
    assert rel_err(a, ref).max() <= TOL
    sizes = [0, 1, 900, 130, 2, 2100, 64]
    mols, coords, types, off = _ensemble(sizes, seed=4100, nq=nq)
    c = torch.from_numpy(coords).cuda()
    t = torch.from_numpy(types).cuda()
    tab = torch.from_numpy(mols[0].table).cuda()
    a = sd.debye_profile_batched(c, t, off, tab, mols[0].q, ctx=grid_ctx).cpu().numpy()
    b = sd.debye_profile_batched(c, t, off, tab, mols[0].q, ctx=pers_ctx).cpu().numpy()
    assert pers_ctx.launch() == "persistent"
    assert np.array_equal(a, b)
    d = sd.debye_profile_batched(c, t, off, tab, mols[0].q, ctx=auto_ctx).cpu().numpy()
    assert auto_ctx.launch() == "grid" and np.array_equal(a, d)
    with pytest.raises(sd.SasError) as e:
        auto_ctx.set_form("persistent+grid")
    assert e.value.status == 1


def test_plan_reuses_tuned_shape(sd):
    import torch

    say("batched plan: second plan of the same workload reuses the tuned shape")
    sizes = [300, 1200, 77]
    mols, coords, types, off = _ensemble(sizes, seed=3100, nq=25)
    ctx = sd.Context(0)
    c = torch.from_numpy(coords).cuda()
    t = torch.from_numpy(types).cuda()
    tab = torch.from_numpy(mols[0].table).cuda()
    p1 = sd.BatchedPlan(c, t, off, tab, mols[0].q, ctx=ctx)
    a = p1.execute().clone()
    v1 = ctx.variant()
    p2 = sd.BatchedPlan(c, t, off, tab, mols[0].q, ctx=ctx)
    b = p2.execute().clone()
    torch.cuda.synchronize()
    assert ctx.variant() == v1
    assert torch.equal(a, b)
    p1.close()
    p2.close()


def test_full_ensemble_plan_against_oracle(sd):
    """The batching workload at full size: 256 globular structures of 500 to
    8,000 atoms on 100 q over [0, 0.8], as one plan (tuned tile shape,
    largest-first order, captured graph) replayed twice with eager work in
    between.  Eight members (the largest, the smallest and six drawn with a
    fixed seed) against their stored oracle profiles at every q; all 256
    bitwise against plain calls with the plan's tile shape."""
    import torch

    from tests.golden.make_golden import ensemble_members, load_ensemble

    say("full ensemble: 256 structures, plan replay vs stored oracle members and plain calls")
    e = W.globular_ensemble()
    gold = load_ensemble()
    assert sorted(gold) == sorted(ensemble_members(e.sizes))
    c = torch.from_numpy(e.coords).cuda()
    t = torch.from_numpy(e.types).cuda()
    tab = torch.from_numpy(e.table).cuda()
    ctx = sd.Context(0)
    plan = sd.BatchedPlan(c, t, e.offsets, tab, e.q, ctx=ctx)
    first = plan.execute().clone()
    bj, qc = ctx.variant()
    ctx2 = sd.Context(0)
    ctx2.set_variant(bj, qc)
    eager = sd.debye_profile_batched(c, t, e.offsets, tab, e.q, ctx=ctx2)
    second = plan.execute().clone()
    torch.cuda.synchronize()
    assert torch.equal(first, second) and torch.equal(first, eager)
    got = second.cpu().numpy()
    worst = 0.0
    for s, (q, I, _) in gold.items():
        assert np.array_equal(q, e.q)
        err = rel_err(got[s], I)
        worst = max(worst, float(err.max()))
        assert err.max() <= TOL, f"structure {s} (N={int(e.sizes[s])}): max rel err {err.max():.3e}"
    print(f"tile shape bj={bj} qc={qc}; stored members: max rel err {worst:.3e}")
    for s in range(len(e.sizes)):
        a, b = int(e.offsets[s]), int(e.offsets[s + 1])
        plain = sd.debye_profile(c[a:b], t[a:b], tab, e.q, ctx=ctx2)
        assert torch.equal(second[s], plain), f"structure {s}"
    plan.close()
