"""The one-shot entry point dom_agg_run (records carry the weights) against
the oracle, element by element, and against plan + forward."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import DEV, check_exact, check_fp, expected, to_dev

pytestmark = pytest.mark.gpu


def _run(c, w, op, **kw):
    from paper_2305_16751_amd import dom_agg_run
    return dom_agg_run(to_dev(c.D), to_dev(c.Q), None if w is None else to_dev(w), op, **kw)


OPS = [("sum", np.int32), ("max", np.int32), ("count", None), ("sum", np.float32), ("max", np.float32),
       ("sum", np.int64), ("max", np.float64)]


@pytest.mark.parametrize("m,coord,alpha", [(1, "int", 1000), (2, "int", 6), (2, "int", 1 << 20), (2, "f32", None),
                                           (3, "int", 1 << 20), (3, "f32", 16), (4, "int", 1000),
                                           (4, "f32", None)])
def test_run_matches_oracle(m, coord, alpha):
    n = {1: 3000, 2: 2500, 3: 900, 4: 300}[m]
    c = workloads.small_case(500 + m * 11 + (alpha or 0) % 97, m, n, n - 19, alphabet=alpha, coord=coord,
                             weight="int64")
    for op, wdt in OPS:
        w = None if wdt is None else (c.w.astype(wdt) if np.dtype(wdt).kind == "i"
                                      else (c.w.astype(np.float64) * 0.37 - 100.0).astype(wdt))
        got = _run(c, w, op)
        what = f"m={m} {coord} {op} {wdt}"
        if op == "sum" and np.dtype(wdt).kind == "f":
            w64 = w.astype(np.float64)
            check_fp(got, oracle.construction(m, c.D, c.Q, w64, "sum"),
                     oracle.construction(m, c.D, c.Q, np.abs(w64), "sum"), what)
        else:
            check_exact(got, expected(m, c.D, c.Q, w, op, wdt), what)


@pytest.mark.parametrize("m", [2, 3])
def test_run_equals_plan_forward_bit_for_bit(m):
    """Same records, same order, same scan tiles: identical fp32 sums.  Both
    paths run untuned (they are tuned separately, and the scan's tile shape
    decides the summation order) on keys of at most 24 bits (wider keys take
    64 bits in the one-shot records, whose scan then uses smaller tiles)."""
    from paper_2305_16751_amd import DomAggPlan
    n, alpha = (60000, None) if m == 2 else (8000, 4096)
    c = workloads.small_case(600 + m, m, n, n, alphabet=alpha, coord="f32", weight="f32")
    p = DomAggPlan(to_dev(c.D), to_dev(c.Q), tune=False)
    assert p.info()["key_bits"] <= 24
    b = p.forward(to_dev(c.w), "sum").cpu().numpy()
    a = _run(c, c.w, "sum", tune=False).cpu().numpy()
    assert np.array_equal(a, b)


def test_run_with_wide_keys():
    """m = 3 with 13-digit ranks on both expanded axes: the 26-bit key leaves
    no room for the query flag in 32 bits, so the records use 64-bit keys."""
    from paper_2305_16751_amd import DomAggPlan
    c = workloads.small_case(610, 3, 7000, 7000, alphabet=1 << 20, coord="int", weight="int64")
    kb = DomAggPlan(to_dev(c.D), to_dev(c.Q)).info()["key_bits"]
    assert 24 < kb <= 32, kb
    check_exact(_run(c, c.w.astype(np.int32), "sum"), expected(3, c.D, c.Q, c.w.astype(np.int32), "sum", np.int32),
                "wide sum")
    check_exact(_run(c, None, "count"), expected(3, c.D, c.Q, None, "count"), "wide count")


@pytest.mark.parametrize("m", [1, 2])
def test_run_batched_with_empty_instances(m):
    rng = np.random.default_rng(61 + m)
    sizes_d = [0, 5, 300, 1, 0, 700, 64, 2]
    sizes_q = [3, 0, 250, 0, 9, 650, 65, 1]
    Ds = [rng.integers(0, 50 + 40 * k, size=(nd, m), dtype=np.int32) for k, nd in enumerate(sizes_d)]
    Qs = [rng.integers(0, 50 + 40 * k, size=(nq, m), dtype=np.int32) for k, nq in enumerate(sizes_q)]
    ws = [rng.standard_normal(nd).astype(np.float32) for nd in sizes_d]
    doff = np.concatenate([[0], np.cumsum(sizes_d)]).astype(np.int64)
    qoff = np.concatenate([[0], np.cumsum(sizes_q)]).astype(np.int64)
    c = workloads.Case("batch", m, np.concatenate(Ds), np.concatenate(Qs), np.concatenate(ws))
    out = _run(c, c.w, "sum", d_offsets=doff, q_offsets=qoff).cpu().numpy()
    mx = _run(c, c.w, "max", d_offsets=doff, q_offsets=qoff).cpu().numpy()
    for k in range(len(sizes_d)):
        if not sizes_q[k]:
            continue
        w64 = ws[k].astype(np.float64)
        check_fp(torch.from_numpy(out[qoff[k]:qoff[k + 1]]), oracle.construction(m, Ds[k], Qs[k], w64, "sum"),
                 oracle.construction(m, Ds[k], Qs[k], np.abs(w64), "sum"), f"instance {k}")
        check_exact(torch.from_numpy(mx[qoff[k]:qoff[k + 1]]), oracle.construction(m, Ds[k], Qs[k], w64, "max"),
                    f"instance {k} max")


def test_run_empty_sides():
    from paper_2305_16751_amd import dom_agg_run
    q = to_dev(np.random.default_rng(0).random((50, 2), dtype=np.float32))
    d0 = torch.empty((0, 2), dtype=torch.float32, device=DEV)
    assert dom_agg_run(d0, q, torch.empty(0, device=DEV), "sum").abs().max().item() == 0
    assert (dom_agg_run(d0, q, None, "count") == 0).all()
    assert dom_agg_run(q, d0, torch.ones(50, device=DEV), "sum").numel() == 0
