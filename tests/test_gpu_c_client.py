"""The C ABI used from plain C (tests/c_client/sas_client.c, built by
__graft_entry__.build()): a profile computed by a C program matches the FP64
oracle, and the program's error-path checks pass."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

CLIENT = os.path.join(os.path.dirname(__file__), "c_client", "sas_client")


@pytest.mark.parametrize("n,nq", [(1, 5), (777, 41), (3000, 100)])
def test_c_client_profile(tmp_path, n, nq):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(CLIENT), "build the C client first (__graft_entry__.build())"
    m = W.random_molecule(1500 + n, n, nq, t=4, q0=0.0, q1=1.0, extent=3.0 * n ** (1 / 3) + 2.0)
    src = tmp_path / "in.bin"
    dst = tmp_path / "out.bin"
    with open(src, "wb") as fh:
        fh.write(np.int64(m.n).tobytes())
        fh.write(np.int32(m.table.shape[0]).tobytes())
        fh.write(np.int32(len(m.q)).tobytes())
        fh.write(np.ascontiguousarray(m.coords, dtype=np.float32).tobytes())
        fh.write(np.ascontiguousarray(m.types, dtype=np.int32).tobytes())
        fh.write(np.ascontiguousarray(m.table, dtype=np.float32).tobytes())
        fh.write(np.ascontiguousarray(m.q, dtype=np.float64).tobytes())
    print(f"[case] C client N={n} Nq={nq}", flush=True)
    r = subprocess.run([CLIENT, str(src), str(dst)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, (r.returncode, r.stderr)
    got = np.fromfile(dst, dtype=np.float64)
    ref = oracle.profile(m.coords, m.types, m.table, m.q)
    assert np.max(np.abs(got - ref) / ref) <= 1e-6
