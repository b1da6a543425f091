"""HIP path vs the CPU oracle, element by element, on seeded inputs.

Every call goes through the C-ABI (via the ctypes front end).  Integer F and
max are compared bit-exactly; fp32 sums per query within
2e-6 * (sum of |w| over the dominated data points), against fp64.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import DEV, check_exact, check_fp, expected, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2305_16751_amd import binding
    binding.load()
    assert torch.cuda.is_available()


def _plan(c, **kw):
    from paper_2305_16751_amd import DomAggPlan
    return DomAggPlan(to_dev(c.D), to_dev(c.Q), **kw)


def _run_and_check(c, op, wdtype, **plan_kw):
    plan = _plan(c, **plan_kw)
    w = None if op == "count" else c.w.astype(wdtype)
    out = plan.forward(None if w is None else to_dev(w), op)
    want, E, L = oracle.construction(c.m, c.D, c.Q, None if w is None else
                                     w.astype(np.float64 if np.dtype(wdtype).kind == "f" else np.int64),
                                     op, weight_dtype=wdtype if w is not None else None, return_stats=True)
    info = plan.info()
    assert info["records"] == E, (info["records"], E)
    assert info["L"] == L, (info["L"], L)
    if op == "sum" and np.dtype(wdtype).kind == "f":
        scale = oracle.construction(c.m, c.D, c.Q, np.abs(w.astype(np.float64)), "sum")
        check_fp(out, want, scale, f"{c.name} {op} {wdtype}")
    else:
        check_exact(out, want, f"{c.name} {op} {wdtype}")
    return plan, out


# ---------------------------------------------------------------------------
# worked example


def test_worked_example(golden_dir):
    import os
    rows = {}
    for line in open(os.path.join(golden_dir, "worked_example_2d.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split(":", 1)
            rows[k.strip()] = v.split()
    D = np.array([s.split(",") for s in rows["D"]], dtype=np.int32)
    Q = np.array([s.split(",") for s in rows["Q"]], dtype=np.int32)
    w = np.array(rows["w"], dtype=np.int64)
    c = workloads.Case("worked", 2, D, Q, w)
    plan = _plan(c)
    assert plan.info()["records"] == int(rows["E"][0])
    check_exact(plan.forward(to_dev(w), "sum"), np.array(rows["sum"], dtype=np.int64), "sum")
    check_exact(plan.forward(None, "count"), np.array(rows["count"], dtype=np.int64), "count")
    mx = plan.forward(to_dev(w.astype(np.float32)), "max").cpu().numpy()
    np.testing.assert_array_equal(mx, np.array(rows["max"], dtype=np.float32))


# ---------------------------------------------------------------------------
# small random inputs with heavy ties, every m / op / dtype


CASES = []
for m in (1, 2, 3, 4):
    for coord, alpha in (("int", 6), ("int", 1000), ("f32", 16), ("f32", None)):
        CASES.append((m, coord, alpha))


@pytest.mark.parametrize("m,coord,alpha", CASES)
def test_small_int_weights(m, coord, alpha):
    n = {1: 3000, 2: 2500, 3: 900, 4: 300}[m]
    c = workloads.small_case(100 + m * 7 + (alpha or 0), m, n, n - 37, alphabet=alpha, coord=coord, weight="int64")
    plan, _ = _run_and_check(c, "sum", np.int64)
    want = expected(m, c.D, c.Q, None, "count")
    check_exact(plan.forward(None, "count"), want, "count")
    check_exact(plan.forward(to_dev(c.w), "max"), expected(m, c.D, c.Q, c.w, "max"), "max i64")
    w32 = c.w.astype(np.int32)
    check_exact(plan.forward(to_dev(w32), "sum"), expected(m, c.D, c.Q, w32, "sum", np.int32), "sum i32")
    check_exact(plan.forward(to_dev(w32), "max"), expected(m, c.D, c.Q, w32, "max", np.int32), "max i32")


@pytest.mark.parametrize("m,coord,alpha", CASES)
def test_small_float_weights(m, coord, alpha):
    n = {1: 3000, 2: 2500, 3: 900, 4: 300}[m]
    c = workloads.small_case(200 + m * 7 + (alpha or 0), m, n - 11, n, alphabet=alpha, coord=coord, weight="f32")
    plan = _plan(c)
    w64 = c.w.astype(np.float64)
    scale = oracle.construction(m, c.D, c.Q, np.abs(w64), "sum")
    check_fp(plan.forward(to_dev(c.w), "sum"), oracle.construction(m, c.D, c.Q, w64, "sum"), scale, "sum f32")
    check_fp(plan.forward(to_dev(w64), "sum"), oracle.construction(m, c.D, c.Q, w64, "sum"), scale, "sum f64",
             tol=1e-12)
    check_exact(plan.forward(to_dev(c.w), "max"), oracle.construction(m, c.D, c.Q, w64, "max"), "max f32")
    check_exact(plan.forward(to_dev(w64), "max"), oracle.construction(m, c.D, c.Q, w64, "max"), "max f64")
    g = np.random.default_rng(m).standard_normal(c.Q.shape[0]).astype(np.float32)
    gw = plan.backward(to_dev(g))
    want = oracle.transposed_sum(m, c.D, c.Q, g.astype(np.float64))
    gs = oracle.transposed_sum(m, c.D, c.Q, np.abs(g.astype(np.float64)))
    check_fp(gw, want, gs, "grad f32")


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 2047, 2048, 2049, 4095, 4096, 4097, 10007])
def test_ragged_sizes(n):
    c = workloads.small_case(n, 2, n, max(n // 2, 1), alphabet=max(n, 4), coord="int", weight="int64")
    _run_and_check(c, "sum", np.int64)


def test_many_tiles_2d_int():
    """Records span hundreds of sort and scan tiles with a ragged tail."""
    c = workloads.small_case(77, 2, 40001, 39999, alphabet=1 << 20, coord="int", weight="int64")
    _run_and_check(c, "sum", np.int64)


# ---------------------------------------------------------------------------
# edge cases


def test_empty_data_and_queries():
    from paper_2305_16751_amd import DomAggPlan
    q = to_dev(np.random.default_rng(0).random((50, 2), dtype=np.float32))
    d0 = torch.empty((0, 2), dtype=torch.float32, device=DEV)
    plan = DomAggPlan(d0, q)
    assert plan.forward(torch.empty(0, device=DEV), "sum").abs().max().item() == 0
    assert (plan.forward(None, "count") == 0).all()
    mx = plan.forward(torch.empty(0, dtype=torch.int32, device=DEV), "max")
    assert (mx == np.iinfo(np.int32).min).all()
    plan2 = DomAggPlan(q, d0)
    assert plan2.forward(torch.ones(50, device=DEV), "sum").numel() == 0
    assert plan2.backward(torch.empty(0, device=DEV)).abs().max().item() == 0


def test_all_points_equal_gives_identity():
    from paper_2305_16751_amd import DomAggPlan
    p = torch.ones((100, 3), dtype=torch.int32, device=DEV)
    plan = DomAggPlan(p, p)
    assert plan.info()["records"] == 0
    assert (plan.forward(torch.ones(100, dtype=torch.int64, device=DEV), "sum") == 0).all()
    mx = plan.forward(torch.ones(100, dtype=torch.float32, device=DEV), "max")
    assert torch.isneginf(mx).all()


def test_nan_coordinate_rejected():
    from paper_2305_16751_amd import DomAggPlan, DomAggError
    d = torch.rand((10, 2), device=DEV)
    d[3, 1] = float("nan")
    with pytest.raises(DomAggError, match="ENAN"):
        DomAggPlan(d, torch.rand((5, 2), device=DEV))


def test_signed_zero_and_infinities():
    D = np.array([[-0.0, 1.0], [0.0, -np.inf], [np.inf, 0.0], [-1.0, -1.0]], dtype=np.float32)
    Q = np.array([[0.0, 2.0], [np.inf, np.inf], [1e-30, 0.5], [-0.0, 3.0]], dtype=np.float32)
    w = np.array([1, 2, 4, 8], dtype=np.int64)
    c = workloads.Case("zeros", 2, D, Q, w)
    _run_and_check(c, "sum", np.int64)


def test_int32_extremes():
    rng = np.random.default_rng(5)
    vals = np.array([np.iinfo(np.int32).min, -1, 0, 1, np.iinfo(np.int32).max], dtype=np.int32)
    D = rng.choice(vals, size=(500, 2)).astype(np.int32)
    Q = rng.choice(vals, size=(400, 2)).astype(np.int32)
    c = workloads.Case("extremes", 2, D, Q, rng.integers(0, 100, 500).astype(np.int64))
    _run_and_check(c, "sum", np.int64)


# ---------------------------------------------------------------------------
# modes


def test_recompute_matches_keep():
    c = workloads.small_case(9, 3, 2000, 1800, alphabet=200, coord="int", weight="int64")
    a = _plan(c).forward(to_dev(c.w), "sum")
    p = _plan(c, recompute=True)
    b = p.forward(to_dev(c.w), "sum")
    check_exact(b, a.cpu().numpy(), "recompute fwd")
    g = np.random.default_rng(1).standard_normal(c.Q.shape[0])
    ga = _plan(c).backward(to_dev(g))
    gb = p.backward(to_dev(g))
    np.testing.assert_allclose(gb.cpu().numpy(), ga.cpu().numpy(), rtol=1e-12, atol=1e-9)


def test_graph_replay_matches_eager():
    c = workloads.small_case(10, 2, 30000, 30000, alphabet=1 << 16, coord="int", weight="int64")
    eager = _plan(c).forward(to_dev(c.w), "sum").cpu().numpy()
    p = _plan(c, graph=True)
    w = to_dev(c.w)
    out = torch.empty(c.Q.shape[0], dtype=torch.int64, device=DEV)
    for r in range(4):
        p.forward(w, "sum", out=out)
        torch.cuda.synchronize()
        check_exact(out, eager, f"replay {r}")
        out.fill_(-7)  # eager work between replays
        torch.cuda.synchronize()


def test_graph_cache_alternating_forward_backward():
    """A training loop alternating forward and backward on one graph plan
    replays one graph per call kind instead of capturing again; every
    replay equals the eager result."""
    c = workloads.small_case(14, 2, 20000, 20000, alphabet=None, coord="f32", weight="f32")
    eager = _plan(c)
    w = to_dev(c.w)
    g = to_dev(np.random.default_rng(2).standard_normal(c.Q.shape[0]).astype(np.float32))
    fe, be = eager.forward(w, "sum").cpu().numpy(), eager.backward(g).cpu().numpy()
    p = _plan(c, graph=True)
    out = torch.empty(c.Q.shape[0], device=DEV)
    gw = torch.empty(c.D.shape[0], device=DEV)
    for r in range(4):
        p.forward(w, "sum", out=out)
        p.backward(g, out=gw)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), fe), f"forward replay {r}"
        assert np.array_equal(gw.cpu().numpy(), be), f"backward replay {r}"
        out.fill_(3.0)  # eager work between replays
        gw.fill_(-3.0)
        torch.cuda.synchronize()
    assert p.info()["graph_captures"] == 2, p.info()


def test_autograd_function():
    from paper_2305_16751_amd import dom_agg
    c = workloads.small_case(11, 2, 3000, 2500, alphabet=None, coord="f32", weight="f32")
    w = to_dev(c.w).requires_grad_(True)
    out = dom_agg(to_dev(c.D), to_dev(c.Q), w, "sum")
    coef = np.random.default_rng(3).standard_normal(c.Q.shape[0]).astype(np.float32)
    (out * to_dev(coef)).sum().backward()
    want = oracle.transposed_sum(2, c.D, c.Q, coef.astype(np.float64))
    scale = oracle.transposed_sum(2, c.D, c.Q, np.abs(coef.astype(np.float64)))
    check_fp(w.grad, want, scale, "autograd grad")


def test_fp32_results_repeat_bit_for_bit():
    """Slot regrouping + left-fold look-back: fp32 sums are run-to-run identical."""
    c = workloads.small_case(12, 2, 60000, 60000, alphabet=None, coord="f32", weight="f32")
    p = _plan(c)
    assert p.info()["regroup_slots"] > 0
    w = to_dev(c.w)
    g = to_dev(np.random.default_rng(8).standard_normal(c.Q.shape[0]).astype(np.float32))
    a = p.forward(w, "sum").cpu().numpy()
    ga = p.backward(g).cpu().numpy()
    for _ in range(3):
        assert np.array_equal(p.forward(w, "sum").cpu().numpy(), a)
        assert np.array_equal(p.backward(g).cpu().numpy(), ga)
    q = _plan(c)  # a second plan of the same points
    assert np.array_equal(q.forward(w, "sum").cpu().numpy(), a)


def test_compact_regroup_path_m4():
    """Wide ranks in m = 4 make the level-tuple table sparse: the plan uses
    the compact table (one place per record), which must give the same
    results, and fp32 sums that repeat bit for bit."""
    c = workloads.small_case(13, 4, 4000, 4000, alphabet=None, coord="f32", weight="int64")
    p = _plan(c)
    assert p.info()["regroup_slots"] == 0, p.info()
    want = oracle.construction(4, c.D, c.Q, c.w, "sum")
    check_exact(p.forward(to_dev(c.w), "sum"), want, "compact sum")
    check_exact(p.forward(to_dev(c.w), "max"), oracle.construction(4, c.D, c.Q, c.w, "max"), "compact max")
    check_exact(p.forward(None, "count"), oracle.construction(4, c.D, c.Q, None, "count"), "compact count")
    wf = c.w.astype(np.float32)
    g = np.random.default_rng(9).standard_normal(c.Q.shape[0]).astype(np.float32)
    gw = p.backward(to_dev(g))
    check_fp(gw, oracle.transposed_sum(4, c.D, c.Q, g.astype(np.float64)),
             oracle.transposed_sum(4, c.D, c.Q, np.abs(g.astype(np.float64))), "compact grad")
    fw = p.forward(to_dev(wf), "sum")
    check_fp(fw, oracle.construction(4, c.D, c.Q, wf.astype(np.float64), "sum"),
             oracle.construction(4, c.D, c.Q, np.abs(wf.astype(np.float64)), "sum"), "compact f32 sum")
    a, ga = fw.cpu().numpy(), gw.cpu().numpy()
    for _ in range(3):
        assert np.array_equal(p.forward(to_dev(wf), "sum").cpu().numpy(), a)
        assert np.array_equal(p.backward(to_dev(g)).cpu().numpy(), ga)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_compact_layout_forced(m, monkeypatch):
    """DOM_AGG_COMPACT=1 puts m <= 3 plans on the compact regroup layout
    (one place per query record) that sparse m = 4 tables use: same results
    on forward (sum, max, count), backward and a batch."""
    monkeypatch.setenv("DOM_AGG_COMPACT", "1")
    n = {1: 5000, 2: 6000, 3: 1500}[m]
    c = workloads.small_case(1400 + m, m, n, n - 77, alphabet=None, coord="f32", weight="int64")
    p = _plan(c)
    assert p.info()["regroup_slots"] == (1 if m == 1 else 0), p.info()
    check_exact(p.forward(to_dev(c.w), "sum"), oracle.construction(m, c.D, c.Q, c.w, "sum"), "sum")
    check_exact(p.forward(to_dev(c.w), "max"), oracle.construction(m, c.D, c.Q, c.w, "max"), "max")
    check_exact(p.forward(None, "count"), oracle.construction(m, c.D, c.Q, None, "count"), "count")
    g = np.random.default_rng(10 + m).standard_normal(c.Q.shape[0]).astype(np.float32)
    check_fp(p.backward(to_dev(g)), oracle.transposed_sum(m, c.D, c.Q, g.astype(np.float64)),
             oracle.transposed_sum(m, c.D, c.Q, np.abs(g.astype(np.float64))), "grad")
    from paper_2305_16751_amd import DomAggPlan
    rng = np.random.default_rng(1450 + m)
    sizes = [700, 0, 1100, 5]
    Ds = [rng.integers(0, 50, size=(k, m), dtype=np.int32) for k in sizes]
    Qs = [rng.integers(0, 50, size=(k + 3, m), dtype=np.int32) for k in sizes]
    ws = [rng.integers(-9, 9, size=k).astype(np.int64) for k in sizes]
    off = lambda xs: np.concatenate([[0], np.cumsum([x.shape[0] for x in xs])]).astype(np.int64)
    pb = DomAggPlan(to_dev(np.concatenate(Ds)), to_dev(np.concatenate(Qs)), off(Ds), off(Qs))
    want = np.concatenate([oracle.construction(m, Ds[k], Qs[k], ws[k], "sum") for k in range(len(sizes))])
    check_exact(pb.forward(to_dev(np.concatenate(ws)), "sum"), want, "batched sum")


def test_same_sign_fp32_weights_long_segments():
    """All-positive fp32 weights over segments that span hundreds of scan
    tiles: the error must stay within 2e-6 * sum |w| (compensated sums)."""
    c = workloads.f32_uniform(2, 1 << 20, workloads.BASE_SEED + 41, "pos")
    w = np.abs(c.w).astype(np.float32) + np.float32(0.5)
    p = _plan(c)
    w64 = w.astype(np.float64)
    want = oracle.fenwick2(c.D, c.Q, w64, "sum")
    check_fp(p.forward(to_dev(w), "sum"), want, want, "same-sign sum")
    g = np.full(c.Q.shape[0], 0.75, dtype=np.float32)
    gw = oracle.fenwick2(-c.Q.astype(np.float64), -c.D.astype(np.float64), g.astype(np.float64), "sum")
    check_fp(p.backward(to_dev(g)), gw, gw, "same-sign grad")


# ---------------------------------------------------------------------------
# key-length classes of the record sort, internal numbering in batches


@pytest.mark.parametrize("m,n,alpha", [(2, 20000, 1 << 20), (2, 3000, 300), (3, 6000, 1 << 20), (4, 1500, 1 << 20)])
def test_sort_classes(m, n, alpha):
    """Keys wider than one digit split the record sort into classes; every
    class region must hold exactly its records, sorted."""
    c = workloads.small_case(300 + m, m, n, n + 5, alphabet=alpha, coord="int", weight="int64")
    p, _ = _run_and_check(c, "sum", np.int64)
    info = p.info()
    if info["key_bits"] > 8:
        assert info["sort_classes"] >= 2, info
    assert sum(info["sort_class_records"]) == info["records"], info
    check_exact(p.forward(None, "count"), expected(m, c.D, c.Q, None, "count"), "count")
    # recompute mode rebuilds the records from the stored class sizes
    r = _plan(c, recompute=True)
    check_exact(r.forward(to_dev(c.w), "sum"), oracle.construction(m, c.D, c.Q, c.w, "sum"), "recompute")


@pytest.mark.parametrize("m", [1, 2, 3])
def test_small_batch_with_empty_instances(m):
    """Uneven instances, some without data or queries: per-instance results
    equal separate plans (internal numbering is per instance range)."""
    from paper_2305_16751_amd import DomAggPlan
    rng = np.random.default_rng(40 + m)
    sizes_d = [0, 5, 300, 1, 0, 700, 64, 2]
    sizes_q = [3, 0, 250, 0, 9, 650, 65, 1]
    Ds, Qs, ws = [], [], []
    for k, (nd, nq) in enumerate(zip(sizes_d, sizes_q)):
        Ds.append(rng.integers(0, 50 + 40 * k, size=(nd, m), dtype=np.int32))
        Qs.append(rng.integers(0, 50 + 40 * k, size=(nq, m), dtype=np.int32))
        ws.append(rng.integers(0, 1000, size=nd).astype(np.int64))
    D, Q, w = np.concatenate(Ds), np.concatenate(Qs), np.concatenate(ws)
    doff = np.concatenate([[0], np.cumsum(sizes_d)]).astype(np.int64)
    qoff = np.concatenate([[0], np.cumsum(sizes_q)]).astype(np.int64)
    p = DomAggPlan(to_dev(D), to_dev(Q), doff, qoff)
    out = p.forward(to_dev(w), "sum").cpu().numpy()
    g = rng.standard_normal(Q.shape[0])
    gw = p.backward(to_dev(g)).cpu().numpy()
    for k in range(len(sizes_d)):
        Dk, Qk, wk = Ds[k], Qs[k], ws[k]
        if Qk.shape[0]:
            check_exact(torch.from_numpy(out[qoff[k]:qoff[k + 1]]), oracle.construction(m, Dk, Qk, wk, "sum"),
                        f"instance {k}")
        if Dk.shape[0]:
            want = oracle.transposed_sum(m, Dk, Qk, g[qoff[k]:qoff[k + 1]])
            np.testing.assert_allclose(gw[doff[k]:doff[k + 1]], want, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("m", [2, 3, 4])
def test_batch_key_classes(m):
    """A batch whose instances have different rank widths: the instance id
    sits below the node fields of the record key, the sort reads the node
    fields only (classes by key length, as for one instance), and each
    (tuple, instance) run stays together.  Plan forward, backward and the
    one-shot call (records carrying weights) per instance against the
    oracle."""
    from paper_2305_16751_amd import DomAggPlan, dom_agg_run
    rng = np.random.default_rng(60 + m)
    n = {2: 3000, 3: 800, 4: 250}[m]
    sizes_d = [n, 17, 2 * n, 0, n // 2, 1]
    sizes_q = [n + 1, 0, 2 * n - 5, 4, n // 2, 1]
    alphas = [1 << 20, 6, 300, 50, 1 << 12, 9]
    Ds = [rng.integers(0, a, size=(k, m), dtype=np.int32) for k, a in zip(sizes_d, alphas)]
    Qs = [rng.integers(0, a, size=(k, m), dtype=np.int32) for k, a in zip(sizes_q, alphas)]
    ws = [rng.integers(-500, 500, size=k).astype(np.int64) for k in sizes_d]
    D, Q, w = np.concatenate(Ds), np.concatenate(Qs), np.concatenate(ws)
    doff = np.concatenate([[0], np.cumsum(sizes_d)]).astype(np.int64)
    qoff = np.concatenate([[0], np.cumsum(sizes_q)]).astype(np.int64)
    p = DomAggPlan(to_dev(D), to_dev(Q), doff, qoff)
    info = p.info()
    assert info["sort_classes"] >= 2, info
    assert sum(info["sort_class_records"]) == info["records"], info
    want = np.concatenate([oracle.construction(m, Ds[k], Qs[k], ws[k], "sum") for k in range(len(sizes_d))])
    check_exact(p.forward(to_dev(w), "sum"), want, "batched sum")
    wmax = np.concatenate([oracle.construction(m, Ds[k], Qs[k], ws[k], "max") for k in range(len(sizes_d))])
    check_exact(p.forward(to_dev(w), "max"), wmax, "batched max")
    g = rng.standard_normal(Q.shape[0])
    gw = p.backward(to_dev(g)).cpu().numpy()
    gwant = np.concatenate([oracle.transposed_sum(m, Ds[k], Qs[k], g[qoff[k]:qoff[k + 1]])
                            for k in range(len(sizes_d))])
    np.testing.assert_allclose(gw, gwant, rtol=1e-12, atol=1e-9)
    w32 = w.astype(np.int32)
    got = dom_agg_run(to_dev(D), to_dev(Q), to_dev(w32), "sum", d_offsets=doff, q_offsets=qoff)
    want32 = np.concatenate([oracle.construction(m, Ds[k], Qs[k], ws[k].astype(np.int32).astype(np.int64), "sum",
                                                 weight_dtype=np.int32) for k in range(len(sizes_d))])
    check_exact(got, want32, "batched one-shot sum i32")


# ---------------------------------------------------------------------------
# the flat map's uncached chunks


def test_flat_map_chunks_spanning_many_points():
    """Points that yield at most one record each: data at first-axis ranks
    with at most one 0 digit, queries at ranks with at most one 1 digit
    (Lemma 2's prefix sets, L = 10, every rank present once more so that
    K = 2^10).  A 2048-record chunk then spans more points than the flat map
    caches, so its walk reads them from global memory; the 10-bit node keys
    still split the sort into two classes."""
    from paper_2305_16751_amd import dom_agg_run
    rng = np.random.default_rng(2305)
    L = 10
    K = 1 << L
    dvals = np.array([K - 1] + [(K - 1) ^ (1 << b) for b in range(L)])
    qvals = np.array([0] + [1 << b for b in range(L)])
    nb = 30000
    d0 = np.concatenate([np.arange(K), rng.choice(dvals, nb)])
    q0 = np.concatenate([np.arange(K), rng.choice(qvals, nb)])
    D = np.stack([d0, rng.integers(0, 1 << 20, d0.size)], 1).astype(np.int32)
    Q = np.stack([q0, rng.integers(0, 1 << 20, q0.size)], 1).astype(np.int32)
    w = rng.integers(-1000, 1000, size=D.shape[0]).astype(np.int64)
    c = workloads.Case("many_points_per_chunk", 2, D, Q, w)
    p, _ = _run_and_check(c, "sum", np.int64)
    info = p.info()
    assert info["sort_classes"] >= 2, info
    # at most one record per bulk point: well under 480 points' worth per chunk
    assert info["records"] < 2 * (nb + K * L), info
    # the one-shot entry point (records carrying 4-byte weights)
    w32 = w.astype(np.float32)
    got = dom_agg_run(to_dev(D), to_dev(Q), to_dev(w32), "sum")
    want = oracle.construction(2, D, Q, w32.astype(np.float64), "sum")
    scale = oracle.construction(2, D, Q, np.abs(w32.astype(np.float64)), "sum")
    check_fp(got, want, scale, "one-shot, many points per chunk")
