"""Shared helpers of the GPU parity tests (oracle comparisons, tolerances)."""
from __future__ import annotations

import numpy as np
import torch

import oracle

# fp32 sums: per query, |out - out_fp64| <= TOL * sum over the dominated set of |w|
FP32_TOL = 2e-6
DEV = "cuda:0"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def expected(m, D, Q, w, op, weight_dtype=None):
    """The oracle's construction in fp64 / int64."""
    if op == "count":
        return oracle.construction(m, D, Q, None, "count")
    wd = np.dtype(weight_dtype) if weight_dtype is not None else np.asarray(w).dtype
    ww = np.asarray(w).astype(np.float64 if wd.kind == "f" else np.int64)
    return oracle.construction(m, D, Q, ww, op, weight_dtype=wd)


def check_exact(got: torch.Tensor, want: np.ndarray, what=""):
    g = got.cpu().numpy()
    if g.dtype.kind == "f":
        ok = np.array_equal(g.astype(np.float64), want.astype(np.float64))
    else:
        ok = np.array_equal(g.astype(np.int64), want.astype(np.int64))
    if not ok:
        bad = np.nonzero(g.astype(np.float64) != want.astype(np.float64))[0]
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {bad[:5]}: "
                             f"got {g[bad[:5]]} want {want[bad[:5]]}")


def check_fp(got: torch.Tensor, want: np.ndarray, scale: np.ndarray, what="", tol=FP32_TOL):
    g = got.detach().cpu().numpy().astype(np.float64)
    err = np.abs(g - want)
    lim = tol * scale + 1e-30
    if not np.all(err <= lim):
        i = int(np.argmax(err - lim))
        raise AssertionError(f"{what}: {int((err > lim).sum())} outside tolerance; worst idx {i}: "
                             f"got {g[i]!r} want {want[i]!r} scale {scale[i]!r}")
    return float((err / np.maximum(scale, 1e-300)).max()) if err.size else 0.0
