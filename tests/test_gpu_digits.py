"""The record sort at each digit width (7 and 8 bits, fixed with
DOM_AGG_DIGIT_BITS), with records packed into one word and without
(DOM_AGG_PACK=0): plan forward and backward, the one-shot call (records
carrying their weights) and a batch, each against the oracle element by
element, to the same bar as at the default width."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import check_exact, check_fp, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(params=[(7, "1"), (7, "0"), (8, "1"), (8, "0")], ids=["d7-packed", "d7-split", "d8-packed",
                                                                     "d8-split"])
def width(request, monkeypatch):
    bits, pack = request.param
    monkeypatch.setenv("DOM_AGG_DIGIT_BITS", str(bits))
    monkeypatch.setenv("DOM_AGG_PACK", pack)
    return bits


@pytest.mark.parametrize("m,n,alpha", [(1, 30000, None), (2, 20000, None), (2, 9000, 40), (3, 2500, None),
                                       (4, 500, 30)])
def test_plan_at_width(width, m, n, alpha):
    from paper_2305_16751_amd import DomAggPlan
    c = workloads.small_case(2300 + 7 * m + (alpha or 0), m, n, n - n // 7, alphabet=alpha,
                             coord="f32" if alpha is None else "int", weight="int64")
    print(f"digits {width} m={m} n={n} alpha={alpha}", flush=True)
    p = DomAggPlan(to_dev(c.D), to_dev(c.Q))
    info = p.info()
    assert info["digit_bits"] == width
    want, E, _ = oracle.construction(m, c.D, c.Q, c.w, "sum", weight_dtype=np.int64, return_stats=True)
    assert info["records"] == E
    check_exact(p.forward(to_dev(c.w), "sum"), want, "sum i64")
    wf = (c.w * 0.01).astype(np.float32)
    scale = oracle.construction(m, c.D, c.Q, np.abs(wf.astype(np.float64)), "sum")
    check_fp(p.forward(to_dev(wf), "sum"), oracle.construction(m, c.D, c.Q, wf.astype(np.float64), "sum"),
             scale, "sum f32")
    g = workloads.rng_for(99 + m).standard_normal(c.Q.shape[0]).astype(np.float32)
    gscale = oracle.transposed_sum(m, c.D, c.Q, np.abs(g.astype(np.float64)))
    check_fp(p.backward(to_dev(g)), oracle.transposed_sum(m, c.D, c.Q, g.astype(np.float64)), gscale, "backward")


@pytest.mark.parametrize("m,n", [(2, 20000), (3, 2500)])
def test_oneshot_at_width(width, m, n):
    from paper_2305_16751_amd import dom_agg_run
    c = workloads.small_case(2400 + m, m, n, n + 333, alphabet=None, coord="f32", weight="int64")
    w32 = (c.w % 1000).astype(np.int32)
    out = dom_agg_run(to_dev(c.D), to_dev(c.Q), to_dev(w32), "sum", tune=False)
    check_exact(out, oracle.construction(m, c.D, c.Q, w32.astype(np.int64), "sum", weight_dtype=np.int32),
                "one-shot sum i32")


def test_batched_oneshot_at_width(width):
    """Records carrying their weights in a batch: the query flag sits above
    every digit read at either width, the instance id below them."""
    from paper_2305_16751_amd import dom_agg_run
    rng = np.random.default_rng(2550)
    sizes = [3000, 1, 7000, 0, 250]
    Ds = [rng.random((k, 2), dtype=np.float32) for k in sizes]
    Qs = [rng.random((k + 11, 2), dtype=np.float32) for k in sizes]
    ws = [rng.integers(-300, 300, size=k).astype(np.int32) for k in sizes]
    off = lambda xs: np.concatenate([[0], np.cumsum([x.shape[0] for x in xs])]).astype(np.int64)
    got = dom_agg_run(to_dev(np.concatenate(Ds)), to_dev(np.concatenate(Qs)), to_dev(np.concatenate(ws)), "sum",
                      d_offsets=off(Ds), q_offsets=off(Qs), tune=False)
    want = np.concatenate([oracle.construction(2, Ds[k], Qs[k], ws[k].astype(np.int64), "sum",
                                               weight_dtype=np.int32) for k in range(len(sizes))])
    check_exact(got, want, "batched one-shot sum i32")


def test_batch_at_width(width):
    from paper_2305_16751_amd import DomAggPlan
    rng = np.random.default_rng(2500)
    sizes_d, sizes_q = [4000, 0, 9000, 17], [3500, 60, 0, 12]
    Ds = [rng.integers(0, 200, size=(k, 2), dtype=np.int32) for k in sizes_d]
    Qs = [rng.integers(0, 200, size=(k, 2), dtype=np.int32) for k in sizes_q]
    ws = [rng.integers(-50, 50, size=k).astype(np.int64) for k in sizes_d]
    doff = np.concatenate([[0], np.cumsum(sizes_d)]).astype(np.int64)
    qoff = np.concatenate([[0], np.cumsum(sizes_q)]).astype(np.int64)
    p = DomAggPlan(to_dev(np.concatenate(Ds)), to_dev(np.concatenate(Qs)), doff, qoff)
    assert p.info()["digit_bits"] == width
    want = np.concatenate([oracle.construction(2, Ds[k], Qs[k], ws[k], "sum", weight_dtype=np.int64)
                           for k in range(len(sizes_d))])
    check_exact(p.forward(to_dev(np.concatenate(ws)), "sum"), want, "batched sum")


def test_tuner_caches_width(tmp_path, monkeypatch):
    """The tuner's choice (tile, scan tile, digit width) lands in the cache
    file, one 7-field line per key, and matches what the plan reports."""
    from paper_2305_16751_amd import DomAggPlan
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DOM_AGG_TUNE_CACHE", str(cache))
    monkeypatch.delenv("DOM_AGG_DIGIT_BITS", raising=False)
    c = workloads.small_case(2600, 2, 20000, 18500, alphabet=None, coord="f32", weight="int64")
    p = DomAggPlan(to_dev(c.D), to_dev(c.Q), basic=True)
    info = p.info()
    assert info["digit_bits"] in (7, 8)
    rows = [line.split() for line in cache.read_text().splitlines()]
    assert rows and all(len(r) == 7 for r in rows)
    assert any(int(r[4]) == info["sort_tile"] and int(r[6]) == info["digit_bits"] for r in rows)
    want = oracle.construction_basic(2, c.D, c.Q, c.w, "sum", weight_dtype=np.int64)
    check_exact(p.forward(to_dev(c.w), "sum"), want, "basic sum after tuning")
