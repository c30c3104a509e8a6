"""MI355X (gfx950) Debye summation: Python binding of libsas_debye.so.

The library evaluates the small-angle-scattering profile

    I(q) = sum_k sum_j f_k(q) f_j(q) sin(q r_jk) / (q r_jk)

(Berlin et al., Background section, Eq. 2) with hand-written HIP kernels.
This module only marshals torch tensors (device memory) and the current
torch stream into the C ABI declared in ``include/sas_debye.h``; every step of
the computation runs on the GPU.  There is no CPU fallback: without the built
library or a gfx950 GPU the calls raise.

Tensor conventions
------------------
coords  float32 [N, 3] on the GPU (Angstrom)
types   int32   [N]    on the GPU, values in [0, T)
table   float32 [T, Nq] on the GPU: f_type(q_m)
q       1-D float64 host array / list / CPU tensor (1/Angstrom): finite,
        >= 0, strictly increasing; uniform grids take the recurrence path,
        other grids are evaluated directly
results float64 on the GPU
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import SasError, check, load

__all__ = [
    "Context", "SasError", "q_grid_check", "debye_profile", "debye_profile_noalloc", "debye_profile_batched",
    "debye_grad", "debye_grad_table",
    "debye_profile_hybrid", "orient_degree",
    "BatchedPlan", "DebyeProfile", "debye_profile_autograd", "default_context",
]


def _q_host(q) -> np.ndarray:
    if isinstance(q, torch.Tensor):
        q = q.detach().to("cpu", torch.float64).numpy()
    return np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1))


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def q_grid_check(q) -> tuple[float, float]:
    """(q0, dq) of a uniform grid; raises SasError(SAS_ERR_Q_NOT_UNIFORM) otherwise.
    Host-only: needs the library but no GPU."""
    qh = _q_host(q)
    q0 = ctypes.c_double()
    dq = ctypes.c_double()
    check(load().sas_q_grid_check(qh.ctypes.data_as(ctypes.c_void_p), len(qh), ctypes.byref(q0), ctypes.byref(dq)),
          "sas_q_grid_check")
    return q0.value, dq.value


class Context:
    """A library context on one GPU plus a reusable workspace tensor."""

    def __init__(self, device: int | torch.device | None = None):
        if device is None:
            device = torch.cuda.current_device()
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if dev.type != "cuda":
            raise ValueError("the Debye library runs on a GPU device")
        self.device = torch.device("cuda", dev.index if dev.index is not None else torch.cuda.current_device())
        self._h = ctypes.c_void_p()
        check(load().sas_create(self.device.index, ctypes.byref(self._h)), "sas_create")
        self._ws: Optional[torch.Tensor] = None

    @property
    def handle(self):
        return self._h

    def workspace(self, nbytes: int) -> torch.Tensor:
        """A device byte buffer of at least nbytes, reused across calls on this
        context.  It is not regrown while the current stream is being
        captured into a graph: a captured call would keep writing into the
        buffer the growth releases."""
        nbytes = max(int(nbytes), 256)
        if self._ws is None or self._ws.numel() < nbytes:
            if torch.cuda.is_current_stream_capturing():
                raise RuntimeError(f"the context's workspace must grow to {nbytes} bytes during graph capture: "
                                   "make one call of this size before capturing")
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def set_variant(self, bj: int = 0, qc: int = 0) -> None:
        check(load().sas_set_variant(self._h, bj, qc), "sas_set_variant")

    def variant(self) -> tuple[int, int]:
        bj = ctypes.c_int32()
        qc = ctypes.c_int32()
        check(load().sas_get_variant(self._h, ctypes.byref(bj), ctypes.byref(qc)), "sas_get_variant")
        return bj.value, qc.value

    FORMS = {"auto": 0, "direct": 1, "per_atom": 4, "persistent": 8, "grid": 16}

    def set_form(self, form: str = "auto") -> None:
        """'direct' evaluates every grid by one sine per pair and q;
        'per_atom' weights every pair term by f_j inside the q loop;
        'persistent' and 'grid' force the launch of the recurrence's pair
        kernel (a persistent grid pulling strips from a counter, or one
        work-group per strip; by default single structures use the first);
        'auto' (default) uses the recurrence on uniform grids and chooses
        between the type-sorted and the per-atom form from T and the atom
        counts.  Forms combine with '+' ('direct+per_atom')."""
        flags = 0
        for part in form.split("+"):
            flags |= self.FORMS[part]
        check(load().sas_set_form(self._h, flags), "sas_set_form")

    def form(self) -> str:
        """Form the last profile or gradient call used: 'recurrence' or
        'direct', with '+per_atom' appended for the per-atom form."""
        f = ctypes.c_int()
        check(load().sas_get_form(self._h, ctypes.byref(f)), "sas_get_form")
        return ("direct" if f.value & 1 else "recurrence") + ("+per_atom" if f.value & 4 else "")

    def launch(self) -> str:
        """Launch of the last call's pair kernel: 'persistent' or 'grid'."""
        f = ctypes.c_int()
        check(load().sas_get_form(self._h, ctypes.byref(f)), "sas_get_form")
        return "persistent" if f.value & 8 else "grid"

    def enable_timing(self, on: bool = True) -> None:
        """Bracket every pair-kernel launch with HIP events on its stream."""
        check(load().sas_enable_timing(self._h, int(bool(on))), "sas_enable_timing")

    def read_timing(self) -> dict:
        """Summed device time (ms) and launch counts of the timed pair kernels
        since the last read; waits for the recorded events."""
        f_ms = ctypes.c_double()
        a_ms = ctypes.c_double()
        f_n = ctypes.c_int64()
        a_n = ctypes.c_int64()
        check(load().sas_read_timing(self._h, ctypes.byref(f_ms), ctypes.byref(f_n), ctypes.byref(a_ms),
                                     ctypes.byref(a_n)), "sas_read_timing")
        return {"forward_ms": f_ms.value, "forward_launches": f_n.value, "adjoint_ms": a_ms.value,
                "adjoint_launches": a_n.value}

    def workspace_size(self, n: int, t: int, nq: int, grad: int = 0) -> int:
        """Bytes for a profile (grad 0), coordinate gradient (1) or table gradient (2)."""
        return int(load().sas_debye_workspace_size(self._h, int(n), int(t), int(nq), int(grad)))

    def close(self) -> None:
        if self._h:
            load().sas_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict[int, Context] = {}


def default_context(device: torch.device | int | None = None) -> Context:
    if device is None:
        idx = torch.cuda.current_device()
    else:
        d = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = d.index if d.index is not None else torch.cuda.current_device()
    if idx not in _contexts:
        _contexts[idx] = Context(idx)
    return _contexts[idx]


def _check_inputs(coords: torch.Tensor, types: torch.Tensor, table: torch.Tensor):
    if not (coords.is_cuda and types.is_cuda and table.is_cuda):
        raise ValueError("coords, types and table must be GPU tensors")
    if coords.dtype != torch.float32 or coords.dim() != 2 or coords.shape[1] != 3 or not coords.is_contiguous():
        raise ValueError("coords must be a contiguous float32 [N, 3] tensor")
    if types.dtype != torch.int32 or types.dim() != 1 or types.shape[0] != coords.shape[0] or not types.is_contiguous():
        raise ValueError("types must be a contiguous int32 [N] tensor")
    if table.dtype != torch.float32 or table.dim() != 2 or not table.is_contiguous():
        raise ValueError("table must be a contiguous float32 [T, Nq] tensor")


def debye_profile(coords: torch.Tensor, types: torch.Tensor, table: torch.Tensor, q, *,
                  ctx: Optional[Context] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """I(q_m) for every q_m of the grid (float64 [Nq] on the GPU)."""
    _check_inputs(coords, types, table)
    ctx = ctx or default_context(coords.device)
    qh = _q_host(q)
    n, t, nq = coords.shape[0], table.shape[0], len(qh)
    if table.shape[1] != nq:
        raise ValueError(f"table has {table.shape[1]} columns for {nq} q values")
    if out is None:
        out = torch.empty(nq, dtype=torch.float64, device=coords.device)
    nbytes = ctx.workspace_size(n, t, nq, False)
    ws = ctx.workspace(nbytes)
    check(load().sas_debye_profile(ctx.handle, _ptr(coords), _ptr(types), n, _ptr(table), t,
                                   qh.ctypes.data_as(ctypes.c_void_p), nq, _ptr(out), _ptr(ws), ws.numel(),
                                   _stream(coords.device)), "sas_debye_profile")
    return out


def debye_profile_noalloc(coords: torch.Tensor, types: torch.Tensor, table: torch.Tensor, q, *,
                          ctx: Optional[Context] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """debye_profile through sas_debye_profile_noalloc: no workspace, the
    library's fixed per-GPU scratch instead (uniform q grids; sizes up to its
    SAS_NOALLOC_SCRATCH_BYTES).  Pass ``out`` to allocate nothing at all."""
    _check_inputs(coords, types, table)
    ctx = ctx or default_context(coords.device)
    qh = _q_host(q)
    n, t, nq = coords.shape[0], table.shape[0], len(qh)
    if table.shape[1] != nq:
        raise ValueError(f"table has {table.shape[1]} columns for {nq} q values")
    if out is None:
        out = torch.empty(nq, dtype=torch.float64, device=coords.device)
    check(load().sas_debye_profile_noalloc(ctx.handle, _ptr(coords), _ptr(types), n, _ptr(table), t,
                                           qh.ctypes.data_as(ctypes.c_void_p), nq, _ptr(out),
                                           _stream(coords.device)), "sas_debye_profile_noalloc")
    return out


def _offsets_host(offsets) -> np.ndarray:
    if isinstance(offsets, torch.Tensor):
        offsets = offsets.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(offsets, dtype=np.int64).reshape(-1))


def debye_profile_batched(coords: torch.Tensor, types: torch.Tensor, offsets, table: torch.Tensor, q, *,
                          ctx: Optional[Context] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Profiles of S structures concatenated along the atom axis (rows
    offsets[s]..offsets[s+1]); returns float64 [S, Nq] on the GPU."""
    _check_inputs(coords, types, table)
    ctx = ctx or default_context(coords.device)
    qh = _q_host(q)
    off = _offsets_host(offsets)
    s, t, nq = len(off) - 1, table.shape[0], len(qh)
    if table.shape[1] != nq:
        raise ValueError(f"table has {table.shape[1]} columns for {nq} q values")
    if s < 0 or off[-1] != coords.shape[0]:
        raise ValueError("offsets must end at the number of atoms")
    if out is None:
        out = torch.empty((max(s, 0), nq), dtype=torch.float64, device=coords.device)
    lib = load()
    nbytes = int(lib.sas_debye_workspace_size_batched(ctx.handle, off.ctypes.data_as(ctypes.c_void_p), s, t, nq))
    ws = ctx.workspace(nbytes)
    check(lib.sas_debye_profile_batched(ctx.handle, _ptr(coords), _ptr(types), off.ctypes.data_as(ctypes.c_void_p), s,
                                        _ptr(table), t, qh.ctypes.data_as(ctypes.c_void_p), nq, _ptr(out), _ptr(ws),
                                        ws.numel(), _stream(coords.device)), "sas_debye_profile_batched")
    return out


class BatchedPlan:
    """A batched evaluation bound to fixed buffers; ``execute()`` replays a
    captured graph of the whole launch sequence on the current stream.  The
    caller may rewrite ``coords`` (and ``types``/``table``) in place between
    executions; sizes, offsets and q are fixed."""

    def __init__(self, coords: torch.Tensor, types: torch.Tensor, offsets, table: torch.Tensor, q, *,
                 ctx: Optional[Context] = None):
        _check_inputs(coords, types, table)
        self.ctx = ctx or Context(coords.device)
        self.coords, self.types, self.table = coords, types, table
        self.q = _q_host(q)
        self.offsets = _offsets_host(offsets)
        s, t, nq = len(self.offsets) - 1, table.shape[0], len(self.q)
        self.out = torch.empty((s, nq), dtype=torch.float64, device=coords.device)
        lib = load()
        nbytes = int(lib.sas_debye_workspace_size_batched(self.ctx.handle, self.offsets.ctypes.data_as(ctypes.c_void_p),
                                                          s, t, nq))
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=coords.device)
        self._h = ctypes.c_void_p()
        check(lib.sas_plan_create_batched(self.ctx.handle, _ptr(coords), _ptr(types),
                                          self.offsets.ctypes.data_as(ctypes.c_void_p), s, _ptr(table), t,
                                          self.q.ctypes.data_as(ctypes.c_void_p), nq, _ptr(self.out), _ptr(self.ws),
                                          self.ws.numel(), ctypes.byref(self._h)), "sas_plan_create_batched")

    def execute(self) -> torch.Tensor:
        check(load().sas_plan_execute(self._h, _stream(self.coords.device)), "sas_plan_execute")
        return self.out

    def close(self) -> None:
        if self._h:
            load().sas_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debye_grad(coords: torch.Tensor, types: torch.Tensor, table: torch.Tensor, q, dL_dI: torch.Tensor, *,
               with_profile: bool = False, ctx: Optional[Context] = None):
    """sum_m dL_dI[m] dI(q_m)/dcoords as float64 [N, 3] (and the profile if
    ``with_profile``); any increasing grid (non-uniform ones take the direct
    variant)."""
    _check_inputs(coords, types, table)
    ctx = ctx or default_context(coords.device)
    qh = _q_host(q)
    n, t, nq = coords.shape[0], table.shape[0], len(qh)
    w = dL_dI.detach().to(device=coords.device, dtype=torch.float64).contiguous()
    if w.numel() != nq:
        raise ValueError("dL_dI needs one value per q")
    grad = torch.empty((n, 3), dtype=torch.float64, device=coords.device)
    prof = torch.empty(nq, dtype=torch.float64, device=coords.device) if with_profile else None
    nbytes = ctx.workspace_size(n, t, nq, True)
    ws = ctx.workspace(nbytes)
    check(load().sas_debye_grad(ctx.handle, _ptr(coords), _ptr(types), n, _ptr(table), t,
                                qh.ctypes.data_as(ctypes.c_void_p), nq, _ptr(w), _ptr(grad), _ptr(prof), _ptr(ws),
                                ws.numel(), _stream(coords.device)), "sas_debye_grad")
    return (grad, prof) if with_profile else grad


HYBRID_MODES = {"auto": 0, "orient": 1, "direct": 2}


def orient_degree(q: float, r_max: float, tol: float) -> int:
    """Quadrature degree L the orientation average uses for q, radius and tol."""
    return int(load().sas_orient_degree(float(q), float(r_max), float(tol)))


def debye_profile_hybrid(coords: torch.Tensor, types: torch.Tensor, table: torch.Tensor, q, *, tol: float = 1e-9,
                         mode: str = "auto", ctx: Optional[Context] = None):
    """Profile with the leading q values averaged over orientations where that
    is cheaper than the direct sum (approximate to about ``tol``); returns
    (I float64 [Nq] on the GPU, number of averaged q values).  ``mode``
    "orient" averages every q, "direct" none.  Synchronises the stream once."""
    _check_inputs(coords, types, table)
    ctx = ctx or default_context(coords.device)
    qh = _q_host(q)
    n, t, nq = coords.shape[0], table.shape[0], len(qh)
    md = HYBRID_MODES[mode]
    out = torch.empty(nq, dtype=torch.float64, device=coords.device)
    nbytes = int(load().sas_debye_workspace_size_hybrid(ctx.handle, n, t, nq, md))
    if nbytes == 0:
        check(1, "sas_debye_workspace_size_hybrid")
    ws = ctx.workspace(nbytes)
    n_orient = ctypes.c_int32(0)
    check(load().sas_debye_profile_hybrid(ctx.handle, _ptr(coords), _ptr(types), n, _ptr(table), t,
                                          qh.ctypes.data_as(ctypes.c_void_p), nq, float(tol), md, _ptr(out),
                                          _ptr(ws), ws.numel(), _stream(coords.device), ctypes.byref(n_orient)),
          "sas_debye_profile_hybrid")
    return out, int(n_orient.value)


def debye_grad_table(coords: torch.Tensor, types: torch.Tensor, table: torch.Tensor, q, dL_dI: torch.Tensor, *,
                     with_profile: bool = False, ctx: Optional[Context] = None):
    """dL_dI[m] dI(q_m)/dtable[t][m] as float64 [T, Nq] (and the profile if
    ``with_profile``).  Up to 64 rows the forward pass keeps per-type sums;
    beyond (per-atom form factors), or with the context's form set to
    'per_atom', per-atom sums over all pairs are added by type."""
    _check_inputs(coords, types, table)
    ctx = ctx or default_context(coords.device)
    qh = _q_host(q)
    n, t, nq = coords.shape[0], table.shape[0], len(qh)
    w = dL_dI.detach().to(device=coords.device, dtype=torch.float64).contiguous()
    if w.numel() != nq:
        raise ValueError("dL_dI needs one value per q")
    gt = torch.empty((t, nq), dtype=torch.float64, device=coords.device)
    prof = torch.empty(nq, dtype=torch.float64, device=coords.device) if with_profile else None
    nbytes = ctx.workspace_size(n, t, nq, 2)
    ws = ctx.workspace(nbytes)
    check(load().sas_debye_grad_table(ctx.handle, _ptr(coords), _ptr(types), n, _ptr(table), t,
                                      qh.ctypes.data_as(ctypes.c_void_p), nq, _ptr(w), _ptr(gt), _ptr(prof),
                                      _ptr(ws), ws.numel(), _stream(coords.device)), "sas_debye_grad_table")
    return (gt, prof) if with_profile else gt


class DebyeProfile(torch.autograd.Function):
    """I(q) = DebyeProfile.apply(coords, types, table, q): differentiable with
    respect to ``coords`` (float32 [N, 3]) through the library's adjoint
    kernel (sas_debye_grad) and with respect to ``table`` (float32 [T, Nq],
    any number of rows: per-type sums up to 64 rows, per-atom sums beyond)
    through sas_debye_grad_table."""

    @staticmethod
    def forward(ctx_, coords, types, table, q):
        qh = _q_host(q)
        ctx_.save_for_backward(coords, types, table)
        ctx_.qh = qh
        return debye_profile(coords.detach(), types, table.detach(), qh)

    @staticmethod
    def backward(ctx_, grad_I):
        coords, types, table = ctx_.saved_tensors
        gc = gt = None
        if ctx_.needs_input_grad[0]:
            gc = debye_grad(coords.detach(), types, table.detach(), ctx_.qh, grad_I).to(coords.dtype)
        if ctx_.needs_input_grad[2]:
            gt = debye_grad_table(coords.detach(), types, table.detach(), ctx_.qh, grad_I).to(table.dtype)
        return gc, None, gt, None


def debye_profile_autograd(coords, types, table, q):
    return DebyeProfile.apply(coords, types, table, q)
