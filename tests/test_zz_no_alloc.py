"""dom_agg_run_static (the entry point for callers that cannot allocate)
against dom_agg_run, through the C-ABI: two calls in a row, the second on a
smaller input, results bit for bit equal to dom_agg_run with the tuner off
(same kernels, same tiles), and no allocation through the allocator hook
during the calls.  Inputs too large for the static workspace are rejected
before anything is written."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import DEV, check_exact, check_fp, to_dev

pytestmark = pytest.mark.gpu


def _run(c, w, op, static, out=None, **kw):
    from paper_2305_16751_amd import dom_agg_run
    return dom_agg_run(to_dev(c.D), to_dev(c.Q), None if w is None else to_dev(w), op, tune=False,
                       static=static, out=out, **kw)


@pytest.fixture()
def counting_hook():
    """Routes the library's allocations through a counting hook (backed by
    torch's caching allocator) and restores the front end's hook after."""
    import importlib
    from paper_2305_16751_amd import binding as B
    F = importlib.import_module("paper_2305_16751_amd.dom_agg")  # (the module, not the function)
    lib = F._lib()
    calls = {"alloc": 0, "release": 0}

    def alloc(size, stream, ctx):
        calls["alloc"] += 1
        return F._alloc(size, stream, ctx)

    def release(ptr, stream, ctx):
        calls["release"] += 1
        F._release(ptr, stream, ctx)

    a, r = B.ALLOC_FN(alloc), B.RELEASE_FN(release)
    B.check(lib.dom_agg_set_allocator(a, r, None))
    yield calls
    B.check(lib.dom_agg_set_allocator(F._ALLOC_CB, F._RELEASE_CB, None))


def test_static_matches_run_two_calls(counting_hook):
    torch.cuda.synchronize()
    # first call: m = 2, |D| = |Q| = 2^16 integer points, int32 weights
    c1 = workloads.int2d_64k()
    w1 = c1.w.astype(np.int32)
    print(f"static call 1: m=2 |D|={c1.D.shape[0]} |Q|={c1.Q.shape[0]}", flush=True)
    d1, q1, ww1 = to_dev(c1.D), to_dev(c1.Q), to_dev(w1)
    out1 = torch.empty(c1.Q.shape[0], dtype=torch.int64, device=DEV)
    from paper_2305_16751_amd import dom_agg_run
    before = dict(counting_hook)
    dom_agg_run(d1, q1, ww1, "sum", out=out1, tune=False, static=True)
    torch.cuda.synchronize()
    assert counting_hook == before, (counting_hook, before)
    ref1 = dom_agg_run(d1, q1, ww1, "sum", tune=False).cpu().numpy()
    check_exact(out1, ref1, "static vs run, call 1")
    check_exact(out1, oracle.construction(2, c1.D, c1.Q, w1.astype(np.int64), "sum"), "static vs oracle, call 1")
    # second call, smaller: m = 3 float32 points and weights
    c2 = workloads.small_case(4242, 3, 5000, 4000, alphabet=None, coord="f32", weight="f32")
    print(f"static call 2: m=3 |D|={c2.D.shape[0]} |Q|={c2.Q.shape[0]}", flush=True)
    d2, q2, ww2 = to_dev(c2.D), to_dev(c2.Q), to_dev(c2.w)
    out2 = torch.empty(c2.Q.shape[0], dtype=torch.float32, device=DEV)
    before = dict(counting_hook)
    dom_agg_run(d2, q2, ww2, "sum", out=out2, tune=False, static=True)
    torch.cuda.synchronize()
    assert counting_hook == before, (counting_hook, before)
    ref2 = dom_agg_run(d2, q2, ww2, "sum", tune=False).cpu().numpy()
    assert np.array_equal(out2.cpu().numpy(), ref2), "static vs run, call 2 (fp32 bit for bit)"
    w64 = c2.w.astype(np.float64)
    check_fp(out2, oracle.construction(3, c2.D, c2.Q, w64, "sum"),
             oracle.construction(3, c2.D, c2.Q, np.abs(w64), "sum"), "static vs oracle, call 2")
    # and the first shape again, after the smaller one
    out3 = torch.empty_like(out1)
    dom_agg_run(d1, q1, ww1, "sum", out=out3, tune=False, static=True)
    check_exact(out3, ref1, "static, call 3")


def test_static_count_max_and_batched():
    c = workloads.small_case(4343, 2, 3000, 2500, alphabet=50, coord="int", weight="int64")
    for op, w in (("count", None), ("max", c.w.astype(np.int32)), ("sum", c.w.astype(np.float32))):
        a = _run(c, w, op, True).cpu().numpy()
        b = _run(c, w, op, False).cpu().numpy()
        assert np.array_equal(a, b), op
    doff = np.array([0, 1000, 3000], dtype=np.int64)
    qoff = np.array([0, 2000, 2500], dtype=np.int64)
    w32 = c.w.astype(np.int32)
    a = _run(c, w32, "sum", True, d_offsets=doff, q_offsets=qoff).cpu().numpy()
    b = _run(c, w32, "sum", False, d_offsets=doff, q_offsets=qoff).cpu().numpy()
    assert np.array_equal(a, b)


def test_static_rejects_too_large():
    from paper_2305_16751_amd import DomAggError, dom_agg_run
    c = workloads.f32_uniform(2, 1 << 22, 7, "big")
    d, q, w = to_dev(c.D), to_dev(c.Q), to_dev(c.w)
    out = torch.full((c.Q.shape[0],), 7.0, device=DEV)
    with pytest.raises(DomAggError, match="ETOOBIG"):
        dom_agg_run(d, q, w, "sum", out=out, static=True)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # nothing written
    # and the workspace still serves a call that fits
    small = workloads.small_case(4444, 2, 2000, 2000, alphabet=None, coord="f32", weight="f32")
    a = _run(small, small.w, "sum", True).cpu().numpy()
    b = _run(small, small.w, "sum", False).cpu().numpy()
    assert np.array_equal(a, b)
