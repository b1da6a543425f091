"""PyTorch front end of the dominance aggregation library.

PyTorch provides device memory (the library's workspace comes from torch's
caching allocator) and streams (every call runs on the current stream);
everything else is the HIP library.

    out = dom_agg(d, q, w, op="sum")            # autograd on w for op="sum"
    out = dom_agg_batched(d, q, w, d_off, q_off, op="sum")
    out = dom_agg_run(d, q, w, op="sum")        # one-shot forward (no plan kept)
    plan = DomAggPlan(d, q)                     # coordinate-only phase, reusable
    out = plan.forward(w, "max"); gw = plan.backward(grad_out)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import binding as B

_TORCH_TO_DT = {torch.int32: B.I32, torch.int64: B.I64, torch.float32: B.F32, torch.float64: B.F64}


def _out_dtype(op: str, wdt: torch.dtype | None) -> torch.dtype:
    if op == "count":
        return torch.int64
    if op == "sum" and wdt in (torch.int32, torch.int64):
        return torch.int64
    return wdt


# ---------------------------------------------------------------------------
# torch's caching allocator behind the library's allocation hook

def _alloc(size, stream, ctx):
    try:
        dev = torch.cuda.current_device()
        return torch.cuda.caching_allocator_alloc(int(size), device=dev, stream=int(stream or 0))
    except Exception:  # reported by the library as DOM_AGG_ENOMEM
        return None


def _release(ptr, stream, ctx):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


_ALLOC_CB = B.ALLOC_FN(_alloc)
_RELEASE_CB = B.RELEASE_FN(_release)
_hook_installed = False


def _lib():
    global _hook_installed
    lib = B.load()
    if not _hook_installed:
        # DOM_AGG_TORCH_ALLOC=0 leaves the library on its own allocator (for
        # measurement)
        if os.environ.get("DOM_AGG_TORCH_ALLOC", "1") != "0":
            B.check(lib.dom_agg_set_allocator(_ALLOC_CB, _RELEASE_CB, None))
        _hook_installed = True
    return lib


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


def _coords(x: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if x.dim() != 2:
        raise ValueError(f"{name} must be [n, m]")
    if x.dtype not in (torch.float32, torch.int32):
        raise ValueError(f"{name} must be float32 or int32, got {x.dtype}")
    return x.contiguous()


def _offsets(nD: int, nQ: int, d_offsets, q_offsets):
    if d_offsets is None and q_offsets is None:
        return np.array([0, nD], dtype=np.int64), np.array([0, nQ], dtype=np.int64)
    doff = np.ascontiguousarray(np.asarray(d_offsets, dtype=np.int64))
    qoff = np.ascontiguousarray(np.asarray(q_offsets, dtype=np.int64))
    if doff.shape != qoff.shape or doff.ndim != 1 or doff.size < 2:
        raise ValueError("offsets must be 1-D arrays of equal length n_inst + 1")
    if doff[-1] != nD or qoff[-1] != nQ:
        raise ValueError("offsets must end at the number of rows")
    return doff, qoff


def _weights(w, op: str, nD: int, device):
    if op not in B.OPS:
        raise ValueError(f"op must be one of {list(B.OPS)}")
    if op == "count":
        return None, None
    if w is None or w.device != device or w.shape != (nD,):
        raise ValueError(f"w must be a [{nD}] tensor on {device}")
    if w.dtype not in _TORCH_TO_DT:
        raise ValueError(f"unsupported weight dtype {w.dtype}")
    return w.contiguous(), w.dtype


def _out(out, op: str, wdt, nQ: int, device):
    odt = _out_dtype(op, wdt)
    if out is None:
        return torch.empty(nQ, dtype=odt, device=device)
    if out.dtype != odt or out.shape != (nQ,) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous [{nQ}] {odt} tensor")
    return out


class DomAggPlan:
    """The coordinate-only phase: ranks, flat map and the sorted records.

    d, q: [nD, m] and [nQ, m] float32 or int32 device tensors (same dtype, same
    m).  d_offsets / q_offsets: host int64 [n_inst + 1] for a batch of
    independent instances (rows of instance k: offsets[k] .. offsets[k+1]-1).
    recompute: keep only per-point state and rebuild the records on each
    forward/backward.  graph: replay forward/backward from a HIP graph.
    le_mask: bit a asks for d_a <= q_a on axis a instead of d_a < q_a.
    basic: the basic construction of Sec. 4 (every axis expanded; m <= 3).
    """

    def __init__(self, d: torch.Tensor, q: torch.Tensor, d_offsets=None, q_offsets=None,
                 recompute: bool = False, graph: bool = False, tune: bool = True, le_mask: int = 0,
                 basic: bool = False):
        lib = _lib()
        d = _coords(d, "d")
        q = _coords(q, "q")
        if d.shape[1] != q.shape[1] or d.dtype != q.dtype:
            raise ValueError("d and q must have the same dtype and dimension")
        self.m = int(d.shape[1])
        self.nD, self.nQ = int(d.shape[0]), int(q.shape[0])
        self.device = d.device
        doff, qoff = _offsets(self.nD, self.nQ, d_offsets, q_offsets)
        self.n_inst = int(doff.size - 1)
        flags = ((B.RECOMPUTE if recompute else 0) | (B.GRAPH if graph else 0) | (0 if tune else B.NO_TUNE)
                 | (B.BASIC if basic else 0) | _le_flags(le_mask))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            B.check(lib.dom_agg_plan(ctypes.byref(h), self.m, _TORCH_TO_DT[d.dtype], _ptr(d), _ptr(q),
                                     self.n_inst, doff.ctypes.data_as(ctypes.c_void_p),
                                     qoff.ctypes.data_as(ctypes.c_void_p), flags, _stream()))
        self._h = h
        self._lib = lib

    def info(self) -> dict:
        inf = B.PlanInfo()
        B.check(self._lib.dom_agg_plan_get_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def forward(self, w: torch.Tensor | None = None, op: str = "sum", out: torch.Tensor | None = None):
        w, wdt = _weights(w, op, self.nD, self.device)
        out = _out(out, op, wdt, self.nQ, self.device)
        with torch.cuda.device(self.device):
            B.check(self._lib.dom_agg_forward(self._h, B.OPS[op], _TORCH_TO_DT.get(wdt, B.I64),
                                              _ptr(w) if op != "count" else None, _ptr(out), _stream()))
        return out

    def forward_records(self, w: torch.Tensor | None = None, op: str = "sum"):
        """The final list of Sec. 4: (ids [E] int64, vals [E]), every record in
        nondecreasing ID order (data rows 0..|D|-1, then queries |D|..), each
        with the total of its ID."""
        w, wdt = _weights(w, op, self.nD, self.device)
        E = self.info()["records"]
        ids = torch.empty(E, dtype=torch.int64, device=self.device)
        vals = torch.empty(E, dtype=_out_dtype(op, wdt), device=self.device)
        with torch.cuda.device(self.device):
            B.check(self._lib.dom_agg_forward_records(self._h, B.OPS[op], _TORCH_TO_DT.get(wdt, B.I64),
                                                      _ptr(w) if op != "count" else None, _ptr(ids), _ptr(vals),
                                                      _stream()))
        return ids, vals

    def backward(self, grad_out: torch.Tensor, out: torch.Tensor | None = None):
        if grad_out.dtype not in (torch.float32, torch.float64) or grad_out.shape != (self.nQ,):
            raise ValueError(f"grad_out must be a [{self.nQ}] float32 or float64 tensor")
        g = grad_out.contiguous()
        if out is None:
            out = torch.empty(self.nD, dtype=g.dtype, device=self.device)
        with torch.cuda.device(self.device):
            B.check(self._lib.dom_agg_backward(self._h, _TORCH_TO_DT[g.dtype], _ptr(g), _ptr(out), _stream()))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dom_agg_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DomAggFunction(torch.autograd.Function):
    """out = sum over dominated data of w; grad_w[d] = sum of grad_out[q] over q > d."""

    @staticmethod
    def forward(ctx, w, plan):
        ctx.plan = plan
        ctx.wdtype = w.dtype
        return plan.forward(w, "sum")

    @staticmethod
    def backward(ctx, grad_out):
        return ctx.plan.backward(grad_out.to(ctx.wdtype)), None


def _le_flags(le_mask: int) -> int:
    return sum(B.LE(a) for a in range(4) if (int(le_mask) >> a) & 1)


def dom_agg_run(d: torch.Tensor, q: torch.Tensor, w: torch.Tensor | None = None, op: str = "sum",
                d_offsets=None, q_offsets=None, out: torch.Tensor | None = None, tune: bool = True,
                le_mask: int = 0, basic: bool = False, static: bool = False):
    """One-shot forward (no plan is kept; the records carry the weights).
    static: dom_agg_run_static, which allocates nothing (its workspace is a
    static 256 MiB device array; out must be given or is allocated here)."""
    lib = _lib()
    d = _coords(d, "d")
    q = _coords(q, "q")
    if d.shape[1] != q.shape[1] or d.dtype != q.dtype:
        raise ValueError("d and q must have the same dtype and dimension")
    nD, nQ = int(d.shape[0]), int(q.shape[0])
    doff, qoff = _offsets(nD, nQ, d_offsets, q_offsets)
    w, wdt = _weights(w, op, nD, d.device)
    out = _out(out, op, wdt, nQ, d.device)
    fn = lib.dom_agg_run_static if static else lib.dom_agg_run
    with torch.cuda.device(d.device):
        B.check(fn(int(d.shape[1]), _TORCH_TO_DT[d.dtype], _ptr(d), _ptr(q), int(doff.size - 1),
                                doff.ctypes.data_as(ctypes.c_void_p), qoff.ctypes.data_as(ctypes.c_void_p),
                                B.OPS[op], _TORCH_TO_DT.get(wdt, B.I64), _ptr(w) if op != "count" else None,
                                _ptr(out), (0 if tune else B.NO_TUNE) | (B.BASIC if basic else 0) | _le_flags(le_mask),
                                _stream()))
    return out


def _needs_grad(w, op):
    return op == "sum" and w is not None and w.requires_grad and w.dtype in (torch.float32, torch.float64)


def dom_agg(d: torch.Tensor, q: torch.Tensor, w: torch.Tensor | None = None, op: str = "sum",
            **plan_kwargs) -> torch.Tensor:
    """For every query row of q: F over w[i] of the data rows d[i] strictly
    below it in every coordinate (e when none).  Differentiable in w for
    op="sum" with float weights (a plan is then kept for the backward);
    otherwise one one-shot call."""
    if not _needs_grad(w, op) and not set(plan_kwargs) - {"le_mask", "basic"}:
        return dom_agg_run(d, q, w, op, **plan_kwargs)
    plan = DomAggPlan(d, q, **plan_kwargs)
    if _needs_grad(w, op):
        return DomAggFunction.apply(w, plan)
    return plan.forward(w, op)


def dom_agg_batched(d, q, w, d_offsets, q_offsets, op: str = "sum", **plan_kwargs) -> torch.Tensor:
    """dom_agg over independent instances stacked along the rows."""
    if not _needs_grad(w, op) and not set(plan_kwargs) - {"le_mask", "basic"}:
        return dom_agg_run(d, q, w, op, d_offsets, q_offsets, **plan_kwargs)
    plan = DomAggPlan(d, q, d_offsets, q_offsets, **plan_kwargs)
    if _needs_grad(w, op):
        return DomAggFunction.apply(w, plan)
    return plan.forward(w, op)
