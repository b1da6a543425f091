"""The record sort's digit histograms from each source (DOM_AGG_HIST: the
points in closed form, a pass over the emitted records, the flat map's
per-record loop) on single instances and batches: a wrong count in any bin
would misplace records, so every result is compared with the oracle, bit for
bit on integer weights."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import check_exact, to_dev

pytestmark = pytest.mark.gpu

SOURCES = ["points", "records", "emit"]


def _batch(seed, m, sizes, alphas):
    rng = np.random.default_rng(seed)
    Ds = [rng.integers(0, a, size=(k, m), dtype=np.int32) for k, a in zip(sizes, alphas)]
    Qs = [rng.integers(0, a, size=(k + 7, m), dtype=np.int32) for k, a in zip(sizes, alphas)]
    ws = [rng.integers(-999, 999, size=k).astype(np.int64) for k in sizes]
    off = lambda xs: np.concatenate([[0], np.cumsum([x.shape[0] for x in xs])]).astype(np.int64)
    return Ds, Qs, ws, off(Ds), off(Qs)


@pytest.mark.parametrize("src", SOURCES)
@pytest.mark.parametrize("m,n,le", [(2, 20000, 1), (3, 3000, 0), (3, 2000, 3), (4, 700, 0)])
def test_single_instance(src, m, n, le, monkeypatch):
    from paper_2305_16751_amd import DomAggPlan, dom_agg_run
    monkeypatch.setenv("DOM_AGG_HIST", src)
    c = workloads.small_case(2700 + m + le, m, n, n - 99, alphabet=None, coord="f32", weight="int64")
    print(f"hist {src} m={m} n={n} le={le}", flush=True)
    p = DomAggPlan(to_dev(c.D), to_dev(c.Q), le_mask=le)
    info = p.info()
    want, E, _ = oracle.construction(m, c.D, c.Q, c.w, "sum", weight_dtype=np.int64, return_stats=True,
                                     le_mask=le)
    assert info["records"] == E
    assert sum(info["sort_class_records"]) == E
    check_exact(p.forward(to_dev(c.w), "sum"), want, "plan sum")
    w32 = (c.w % 5000).astype(np.int32)
    got = dom_agg_run(to_dev(c.D), to_dev(c.Q), to_dev(w32), "sum", tune=False, le_mask=le)
    check_exact(got, oracle.construction(m, c.D, c.Q, w32.astype(np.int64), "sum", weight_dtype=np.int32,
                                         le_mask=le), "one-shot sum")


@pytest.mark.parametrize("src", SOURCES)
@pytest.mark.parametrize("m", [2, 3, 4])
def test_batch(src, m, monkeypatch):
    from paper_2305_16751_amd import DomAggPlan
    monkeypatch.setenv("DOM_AGG_HIST", src)
    n = {2: 4000, 3: 900, 4: 300}[m]
    Ds, Qs, ws, doff, qoff = _batch(2800 + m, m, [n, 3, 2 * n, 0, n // 3], [1 << 20, 4, 500, 9, 1 << 10])
    p = DomAggPlan(to_dev(np.concatenate(Ds)), to_dev(np.concatenate(Qs)), doff, qoff)
    want = np.concatenate([oracle.construction(m, Ds[k], Qs[k], ws[k], "sum") for k in range(len(Ds))])
    check_exact(p.forward(to_dev(np.concatenate(ws)), "sum"), want, "batched sum")


@pytest.mark.parametrize("src", SOURCES)
def test_basic_variant_batch(src, monkeypatch):
    """Basic-variant batches keep the instance id among the sorted bits: the
    closed form does not apply and the flat map's histograms are used."""
    from paper_2305_16751_amd import DomAggPlan
    monkeypatch.setenv("DOM_AGG_HIST", src)
    Ds, Qs, ws, doff, qoff = _batch(2900, 2, [1500, 2, 900], [300, 5, 1 << 16])
    p = DomAggPlan(to_dev(np.concatenate(Ds)), to_dev(np.concatenate(Qs)), doff, qoff, basic=True)
    want = np.concatenate([oracle.construction_basic(2, Ds[k], Qs[k], ws[k], "sum") for k in range(len(Ds))])
    check_exact(p.forward(to_dev(np.concatenate(ws)), "sum"), want, "basic batched sum")
