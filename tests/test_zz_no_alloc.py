"""The allocation-free profile call (sas_debye_profile_noalloc) through the C
ABI: its results equal those of sas_debye_profile with a caller workspace,
bit for bit, on two calls in a row (the 50,000-atom, 200-q rod at the
benchmark's shape, then a smaller 1,000-atom, 64-q ellipsoid that reuses the
same scratch), and match the FP64 oracle to 1e-6 per q; it refuses sizes
beyond its fixed scratch and grids that would need an upload; and a capture of
it into a caller's graph replays correctly with eager work between replays."""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_2258_amd as sd
    from paper_1306_2258_amd import _lib

    return sd, _lib.load()


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(m):
    import torch

    return (torch.from_numpy(m.coords).cuda(), torch.from_numpy(m.types).cuda(), torch.from_numpy(m.table).cuda())


def vp(t):
    return ctypes.c_void_p(t.data_ptr())


def call_noalloc(lib, ctx, c, t, tab, q, out, stream):
    qh = np.ascontiguousarray(q, dtype=np.float64)
    return lib.sas_debye_profile_noalloc(ctx.handle, vp(c), vp(t), c.shape[0], vp(tab), tab.shape[0],
                                         qh.ctypes.data_as(ctypes.c_void_p), len(qh), vp(out), stream)


def call_workspace(lib, ctx, c, t, tab, q, out, stream):
    import torch

    qh = np.ascontiguousarray(q, dtype=np.float64)
    nbytes = int(lib.sas_debye_workspace_size(ctx.handle, c.shape[0], tab.shape[0], len(qh), 0))
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
    st = lib.sas_debye_profile(ctx.handle, vp(c), vp(t), c.shape[0], vp(tab), tab.shape[0],
                               qh.ctypes.data_as(ctypes.c_void_p), len(qh), vp(out), vp(ws), ws.numel(), stream)
    return st, ws


def test_two_calls_match_workspace_call_and_oracle(env):
    import torch

    sd, lib = env
    ctx = sd.Context(0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    from tests.golden.make_golden import load

    cases = [(W.dna_rod_50k(), "dna_rod_50k"), (W.ellipsoid_1k(), "ellipsoid_1k")]
    for m, golden in cases:
        say(f"noalloc then workspace call: {m.name} N={m.n} Nq={len(m.q)}")
        c, t, tab = to_dev(m)
        got = torch.full((len(m.q),), float("nan"), dtype=torch.float64, device="cuda")
        want = torch.full((len(m.q),), float("nan"), dtype=torch.float64, device="cuda")
        st = call_noalloc(lib, ctx, c, t, tab, m.q, got, stream)
        assert st == 0, lib.sas_last_error()
        # the workspace call on the tile shape the allocation-free call used
        # (it may take a longer J block to fit its scratch): bitwise equal
        shape = ctx.variant()
        ctx2 = sd.Context(0)
        ctx2.set_variant(shape[0], shape[1])
        st, ws = call_workspace(lib, ctx2, c, t, tab, m.q, want, stream)
        assert st == 0, lib.sas_last_error()
        torch.cuda.synchronize()
        assert ctx2.variant()[:2] == shape[:2]
        assert torch.equal(got, want), f"{m.name}: allocation-free result differs from the workspace call"
        q, I, _ = load(golden)
        assert np.array_equal(q, m.q)
        err = np.abs(got.cpu().numpy() - I) / I
        print(f"{m.name}: max rel err vs oracle {err.max():.3e}", flush=True)
        assert err.max() <= TOL
        del ws


def test_second_call_smaller_than_first(env):
    """A small structure right after a large one: the scratch still holds the
    large call's strip rows; the small call must not read any of them."""
    import torch

    sd, lib = env
    ctx = sd.Context(0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    big = W.random_molecule(7100, 30000, 150, q0=0.0, q1=1.0, extent=60.0)
    small = W.random_molecule(7101, 700, 150, q0=0.0, q1=1.0, extent=18.0)
    outs = []
    for m in (big, small):
        say(f"noalloc {m.name} N={m.n} Nq={len(m.q)}")
        c, t, tab = to_dev(m)
        got = torch.full((len(m.q),), float("nan"), dtype=torch.float64, device="cuda")
        want = torch.full((len(m.q),), float("nan"), dtype=torch.float64, device="cuda")
        assert call_noalloc(lib, ctx, c, t, tab, m.q, got, stream) == 0, lib.sas_last_error()
        shape = ctx.variant()
        ctx2 = sd.Context(0)
        ctx2.set_variant(shape[0], shape[1])
        st, ws = call_workspace(lib, ctx2, c, t, tab, m.q, want, stream)
        assert st == 0, lib.sas_last_error()
        torch.cuda.synchronize()
        assert torch.equal(got, want), m.name
        outs.append(got.cpu().numpy())
        del ws
    ref = oracle.profile(small.coords, small.types, small.table, small.q)
    assert np.max(np.abs(outs[1] - ref) / ref) <= TOL


def test_refusals(env):
    """Host-detected refusals, before any device work: a structure whose
    scratch exceeds the fixed array, a non-uniform grid, the forced direct
    form.  The outputs stay untouched."""
    import torch

    sd, lib = env
    ctx = sd.Context(0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    say("noalloc refusals")
    n = 100000
    c = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    t = torch.zeros(n, dtype=torch.int32, device="cuda")
    q = W.q_grid(0.0, 1.0, 200)
    tab = torch.ones((1, 200), dtype=torch.float32, device="cuda")
    out = torch.full((200,), 7.0, dtype=torch.float64, device="cuda")
    assert call_noalloc(lib, ctx, c, t, tab, q, out, stream) == 3
    msg = lib.sas_last_error().decode()
    assert "bytes of scratch" in msg and str(64 << 20) in msg, msg
    # a forced tile shape is kept: 50,000 atoms fit with J blocks of 512
    # atoms (the automatic choice when the default's rows do not fit), not
    # with a forced 128
    n5 = 50000
    c5 = torch.zeros((n5, 3), dtype=torch.float32, device="cuda")
    t5 = torch.zeros(n5, dtype=torch.int32, device="cuda")
    ctx.set_variant(128, 0)
    assert call_noalloc(lib, ctx, c5, t5, tab, q, out, stream) == 3
    ctx.set_variant(0, 0)
    m = W.random_molecule(7102, 300, 0, q=W.log_grid(1e-3, 0.8, 40), extent=15.0)
    c2, t2, tab2 = to_dev(m)
    out2 = torch.full((40,), 7.0, dtype=torch.float64, device="cuda")
    assert call_noalloc(lib, ctx, c2, t2, tab2, m.q, out2, stream) == 3
    m3 = W.random_molecule(7103, 300, 40, q0=0.0, q1=0.8, extent=15.0)
    c3, t3, tab3 = to_dev(m3)
    ctx.set_form("direct")
    out3 = torch.full((40,), 7.0, dtype=torch.float64, device="cuda")
    assert call_noalloc(lib, ctx, c3, t3, tab3, m3.q, out3, stream) == 3
    ctx.set_form("auto")
    torch.cuda.synchronize()
    assert torch.all(out == 7.0) and torch.all(out2 == 7.0) and torch.all(out3 == 7.0)
    # the same context still computes afterwards
    assert call_noalloc(lib, ctx, c3, t3, tab3, m3.q, out3, stream) == 0
    ref = oracle.profile(m3.coords, m3.types, m3.table, m3.q)
    torch.cuda.synchronize()
    assert np.max(np.abs(out3.cpu().numpy() - ref) / ref) <= TOL


def test_captured_noalloc_call_replays(env):
    """Captured by the caller into a hipGraph (torch.cuda.graph) with nothing
    allocated inside the capture; three replays, each after moving the atoms
    and an eager workspace call, equal that eager result bitwise."""
    import torch

    sd, lib = env
    say("noalloc call captured by torch.cuda.graph, 3 replays")
    m = W.random_molecule(7104, 2500, 100, q0=0.0, q1=1.0, extent=38.0)
    c, t, tab = to_dev(m)
    ctx = sd.Context(0)
    out = torch.empty(len(m.q), dtype=torch.float64, device="cuda")
    want = torch.empty(len(m.q), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            st = call_noalloc(lib, ctx, c, t, tab, m.q, out, ctypes.c_void_p(s.cuda_stream))
    torch.cuda.synchronize()
    assert st == 0, lib.sas_last_error()
    rng = np.random.default_rng(5)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        c.add_(torch.from_numpy(rng.normal(scale=0.05, size=(m.n, 3)).astype(np.float32)).cuda())
        torch.cuda.synchronize()
        st, ws = call_workspace(lib, ctx, c, t, tab, m.q, want, stream)
        assert st == 0
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), f"replay {rep}"
        del ws
    ref = oracle.profile(c.cpu().numpy(), m.types, m.table, m.q)
    assert np.max(np.abs(out.cpu().numpy() - ref) / ref) <= TOL
