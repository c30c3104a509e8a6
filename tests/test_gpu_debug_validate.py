"""The debug mode of the library (SAS_DEBUG_VALIDATE set when a context is
created): device-side checks of type ids and coordinates before each call.

Valid inputs give bitwise the results of the ordinary mode; a type id outside
[0, T) or a non-finite coordinate gives SAS_ERR_INVALID_ARG naming the first
such atom, from every entry point, and leaves the output untouched.  Without
the variable the same inputs are accepted (type ids clamped).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

INVALID_ARG = 1


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


@pytest.fixture
def dbg_ctx(sd, monkeypatch):
    monkeypatch.setenv("SAS_DEBUG_VALIDATE", "1")
    ctx = sd.Context(0)
    monkeypatch.delenv("SAS_DEBUG_VALIDATE")
    return ctx


def _mol(n=300, t=3, nq=40):
    return W.random_molecule(1900 + n, n, nq, t=t, q0=0.0, q1=0.8, extent=15.0)


def _dev(m):
    import torch

    return (torch.from_numpy(m.coords).cuda(), torch.from_numpy(m.types).cuda(), torch.from_numpy(m.table).cuda())


def test_valid_inputs_same_bits(sd, dbg_ctx):
    say("debug mode, valid inputs: bitwise equal to the ordinary mode")
    m = _mol()
    c, t, tab = _dev(m)
    a = sd.debye_profile(c, t, tab, m.q, ctx=dbg_ctx).cpu().numpy()
    b = sd.debye_profile(c, t, tab, m.q, ctx=sd.Context(0)).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("bad", ["type_high", "type_negative", "nan", "inf"])
def test_profile_rejects(sd, dbg_ctx, bad):
    import torch

    say(f"debug mode rejects {bad}")
    m = _mol()
    if bad == "type_high":
        m.types[17] = 3
        first = 17
    elif bad == "type_negative":
        m.types[250] = -1
        m.types[251] = -7
        first = 250
    elif bad == "nan":
        m.coords[4, 1] = np.nan
        first = 4
    else:
        m.coords[299, 2] = np.inf
        first = 299
    c, t, tab = _dev(m)
    out = torch.full((len(m.q),), -5.0, dtype=torch.float64, device="cuda")
    with pytest.raises(sd.SasError) as e:
        sd.debye_profile(c, t, tab, m.q, ctx=dbg_ctx, out=out)
    assert e.value.status == INVALID_ARG
    assert f"atom {first}" in str(e.value)
    assert torch.all(out == -5.0)
    # the ordinary mode accepts the same call
    r = sd.debye_profile(c, t, tab, m.q, ctx=sd.Context(0))
    if bad.startswith("type"):
        assert torch.all(torch.isfinite(r))


def test_every_entry_point_checks(sd, dbg_ctx):
    import torch

    say("debug mode: gradient, table gradient, hybrid, batched and plans check too")
    m = _mol()
    m.types[123] = 9
    c, t, tab = _dev(m)
    w = torch.ones(len(m.q), dtype=torch.float64, device="cuda")
    calls = [
        lambda: sd.debye_grad(c, t, tab, m.q, w, ctx=dbg_ctx),
        lambda: sd.debye_grad_table(c, t, tab, m.q, w, ctx=dbg_ctx),
        lambda: sd.debye_profile_hybrid(c, t, tab, m.q, ctx=dbg_ctx),
        lambda: sd.debye_profile_batched(c, t, [0, 100, 300], tab, m.q, ctx=dbg_ctx),
    ]
    for call in calls:
        with pytest.raises(sd.SasError) as e:
            call()
        assert e.value.status == INVALID_ARG and "atom 123" in str(e.value)
    # a plan checks at every execution: valid at first, then a coordinate
    # rewritten in place to NaN
    m2 = _mol()
    c2, t2, tab2 = _dev(m2)
    plan = sd.BatchedPlan(c2, t2, [0, 120, 300], tab2, m2.q, ctx=dbg_ctx)
    ok = plan.execute().clone()
    ref_ctx = sd.Context(0)
    ref_ctx.set_variant(*dbg_ctx.variant())  # the tile shape the plan's tuning chose
    ref = sd.debye_profile_batched(c2, t2, [0, 120, 300], tab2, m2.q, ctx=ref_ctx)
    assert torch.equal(ok, ref)
    c2[200, 0] = float("nan")
    with pytest.raises(sd.SasError) as e:
        plan.execute()
    assert e.value.status == INVALID_ARG and "atom 200" in str(e.value)
    plan.close()
