"""The HIP path at the full workload sizes, in the launch configuration the
benchmark times (default plan, autotuned tiles), against the oracle's pins.

Every output is checked.  Where the oracle's construction would take
minutes at full size, the pins are independent textbook algorithms with
their own CPU pins (tests/test_oracle*.py): the m = 2 Fenwick sweep
(fp64 sums, exact counts, several weight columns in one pass) and the m = 3
divide and conquer.  fp32 sums are checked per query against fp64 within
2e-6 * (sum of |w| over the dominated set), the scale coming from the same
pin run on |w|.  m = 4 (no textbook pin here) is checked on every instance
at sampled queries and gradient entries against the plain definition.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import DEV, check_exact, check_fp, to_dev

pytestmark = pytest.mark.gpu


def _plan(D, Q, **kw):
    from paper_2305_16751_amd import DomAggPlan
    return DomAggPlan(to_dev(D), to_dev(Q), **kw)


def _sample(n, k, seed):
    rng = np.random.default_rng(seed)
    idx = rng.choice(n, size=min(k, n), replace=False)
    return np.sort(idx)


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_int2d_64k_exact():
    c = workloads.int2d_64k()
    print(f"int2d_64k |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    p = _plan(c.D, c.Q)
    want, E, L = oracle.construction(2, c.D, c.Q, c.w, "sum", return_stats=True)
    assert p.info()["records"] == E and p.info()["L"] == L
    check_exact(p.forward(to_dev(c.w), "sum"), want, "sum")
    check_exact(p.forward(to_dev(c.w), "max"), oracle.construction(2, c.D, c.Q, c.w, "max"), "max")
    cnt = oracle.construction(2, c.D, c.Q, None, "count")
    check_exact(p.forward(None, "count"), cnt, "count")
    np.testing.assert_array_equal(cnt, oracle.fenwick2(c.D, c.Q, None, "count"))
    from paper_2305_16751_amd import dom_agg_run
    check_exact(dom_agg_run(to_dev(c.D), to_dev(c.Q), to_dev(c.w.astype(np.int32)), "sum"), want, "one-shot sum")


def test_f32_2d_2m_every_output():
    """Medium size between the small cases and the full workload: long
    segments (look-back chains over hundreds of tiles)."""
    c = workloads.f32_uniform(2, 1 << 21, workloads.BASE_SEED + 21, "f32_2d_2m")
    print(f"f32_2d_2m |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    p = _plan(c.D, c.Q)
    cnt = p.forward(None, "count").cpu().numpy()
    out = p.forward(to_dev(c.w), "sum")
    g = np.random.default_rng(10).standard_normal(c.Q.shape[0]).astype(np.float32)
    gw = p.backward(to_dev(g))
    w64, g64 = c.w.astype(np.float64), g.astype(np.float64)
    s, sa, n1 = oracle.fenwick2_sums(c.D, c.Q, [w64, np.abs(w64), np.ones_like(w64)])
    np.testing.assert_array_equal(cnt, n1.astype(np.int64))
    check_fp(out, s, sa, "f32_2d_2m sum")
    gs, gsa = oracle.fenwick2_sums(-c.Q.astype(np.float64), -c.D.astype(np.float64), [g64, np.abs(g64)])
    check_fp(gw, gs, gsa, "f32_2d_2m grad")


@pytest.fixture(scope="module")
def c2a():
    """The headline workload (m = 2, |D| = |Q| = 2^24) and the pins of every
    output: fp64 sums of w and |w| and the counts, in one Fenwick pass."""
    c = workloads.f32_2d_16m()
    w64 = c.w.astype(np.float64)
    s, sa, n1 = oracle.fenwick2_sums(c.D, c.Q, [w64, np.abs(w64), np.ones_like(w64)])
    return c, s, sa, n1.astype(np.int64)


def test_f32_2d_16m_plan_forward_every_output(c2a):
    c, s, sa, cnt = c2a
    print(f"f32_2d_16m plan |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    p = _plan(c.D, c.Q)
    out = p.forward(to_dev(c.w), "sum").cpu()
    got_cnt = p.forward(None, "count").cpu().numpy()
    # same-sign weights over segments of ~4000 scan tiles (compensated fp32)
    pos = p.forward(to_dev(np.abs(c.w)), "sum").cpu()
    del p
    _free()
    np.testing.assert_array_equal(got_cnt, cnt)
    check_fp(out, s, sa, "f32_2d_16m plan sum")
    check_fp(pos, sa, sa, "f32_2d_16m plan sum of |w|")


def test_f32_2d_16m_one_shot_every_output(c2a):
    """The one-shot entry point the benchmark times (records carry the
    weights)."""
    from paper_2305_16751_amd import dom_agg_run
    c, s, sa, cnt = c2a
    print(f"f32_2d_16m one-shot |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    d, q = to_dev(c.D), to_dev(c.Q)
    out = dom_agg_run(d, q, to_dev(c.w), "sum").cpu()
    got_cnt = dom_agg_run(d, q, None, "count").cpu().numpy()
    pos = dom_agg_run(d, q, to_dev(np.abs(c.w)), "sum").cpu()
    del d, q
    _free()
    np.testing.assert_array_equal(got_cnt, cnt)
    check_fp(out, s, sa, "f32_2d_16m one-shot sum")
    check_fp(pos, sa, sa, "f32_2d_16m one-shot sum of |w|")


def test_f32_3d_1m_every_output():
    from paper_2305_16751_amd import dom_agg_run
    c = workloads.f32_3d_1m()
    print(f"f32_3d_1m |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    p = _plan(c.D, c.Q)
    out = p.forward(to_dev(c.w), "sum").cpu()
    cnt = p.forward(None, "count").cpu().numpy()
    one = dom_agg_run(to_dev(c.D), to_dev(c.Q), to_dev(c.w), "sum").cpu()
    del p
    _free()
    w64 = c.w.astype(np.float64)
    np.testing.assert_array_equal(cnt, oracle.sweep(3, c.D, c.Q, None, "count"))
    want = oracle.sweep(3, c.D, c.Q, w64, "sum")
    scale = oracle.sweep(3, c.D, c.Q, np.abs(w64), "sum")
    check_fp(out, want, scale, "f32_3d_1m sum")
    check_fp(one, want, scale, "f32_3d_1m one-shot sum")


def _brute_grad_2d(D, Q, c, idx):
    """The definition of the gradient at the data points idx, in fp64:
    sum of c over the queries strictly above D[i] on both axes (queries
    sorted by the first axis once; per point, the candidates right of it are
    filtered on the second axis)."""
    order = np.argsort(Q[:, 0], kind="stable")
    qx = Q[order, 0].astype(np.float64)
    qy = Q[order, 1].astype(np.float64)
    cc = c[order].astype(np.float64)
    out = np.empty(idx.size)
    aout = np.empty(idx.size)
    for k, i in enumerate(idx):
        lo = np.searchsorted(qx, np.float64(D[i, 0]), side="right")
        sel = qy[lo:] > np.float64(D[i, 1])
        out[k] = cc[lo:][sel].sum()
        aout[k] = np.abs(cc[lo:][sel]).sum()
    return out, aout


def test_f32_2d_4m_grad():
    """Forward + adjoint: every forward output and every gradient entry
    against the Fenwick pin (the gradient is the transposed dominance sum,
    a sweep on (-Q weighted by c, -D)); the gradient also against the fp64
    definition on a 4096-point subset and against central finite
    differences of the fp64 loss."""
    from paper_2305_16751_amd import dom_agg, DomAggPlan
    c = workloads.f32_2d_4m_grad()
    print(f"f32_2d_4m_grad |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    d, q = to_dev(c.D), to_dev(c.Q)
    w = to_dev(c.w).requires_grad_(True)
    out = dom_agg(d, q, w, "sum")
    loss = (out * to_dev(c.c)).sum()
    loss.backward()
    grad = w.grad.cpu().numpy().astype(np.float64)
    w64, c64 = c.w.astype(np.float64), c.c.astype(np.float64)
    s, sa = oracle.fenwick2_sums(c.D, c.Q, [w64, np.abs(w64)])
    check_fp(out.detach(), s, sa, "forward")
    gs, gsa = oracle.fenwick2_sums(-c.Q.astype(np.float64), -c.D.astype(np.float64), [c64, np.abs(c64)])
    check_fp(torch.from_numpy(grad), gs, gsa, "grad vs sweep (every entry)")
    di = _sample(c.D.shape[0], 4096, 3)
    want, scale = _brute_grad_2d(c.D, c.Q, c.c, di)
    check_fp(torch.from_numpy(grad[di]), want, scale, "grad vs definition (4096 points)")
    # finite differences of the fp64 loss (the GPU path with float64 weights)
    plan = DomAggPlan(d, q)
    wd = to_dev(w64)
    cq = to_dev(c64)
    rng = np.random.default_rng(4)
    v = np.zeros(c.D.shape[0])
    v[di] = rng.standard_normal(di.size)
    vd = to_dev(v)
    eps = 1e-3
    lp = float((plan.forward(wd + eps * vd, "sum") * cq).sum())
    lm = float((plan.forward(wd - eps * vd, "sum") * cq).sum())
    fd = (lp - lm) / (2 * eps)
    gv = float(grad @ v)
    assert abs(fd - gv) <= 1e-4 * (abs(gv) + np.abs(grad[di]) @ np.abs(v[di])), (fd, gv)
    for i in di[:16]:
        e = torch.zeros(c.D.shape[0], dtype=torch.float64, device=DEV)
        e[int(i)] = eps
        fdi = (float((plan.forward(wd + e, "sum") * cq).sum()) - float((plan.forward(wd - e, "sum") * cq).sum())) / (2 * eps)
        assert abs(fdi - grad[i]) <= 1e-4 * (abs(grad[i]) + 1.0), (int(i), fdi, grad[i])


def _separate_instances(c):
    """One m = 2 problem equal to the batch: instance k's points move by
    (+k B, -k B), B above every coordinate span, so that no point of one
    instance dominates a point of another (exact in fp64 for these
    integers)."""
    B = float(1 << 17)
    kd = np.repeat(np.arange(len(c.d_offsets) - 1), np.diff(c.d_offsets)).astype(np.float64)
    kq = np.repeat(np.arange(len(c.q_offsets) - 1), np.diff(c.q_offsets)).astype(np.float64)
    D = c.D.astype(np.float64) + np.stack([kd * B, -kd * B], 1)
    Q = c.Q.astype(np.float64) + np.stack([kq * B, -kq * B], 1)
    return D, Q


def test_batched_int2d_every_instance():
    from paper_2305_16751_amd import DomAggPlan
    c = workloads.batched_int2d()
    print(f"batched_int2d instances={len(c.d_offsets) - 1} points={c.n}", flush=True)
    d, q, w = to_dev(c.D), to_dev(c.Q), to_dev(c.w)
    pb = DomAggPlan(d, q, c.d_offsets, c.q_offsets, graph=True)
    outb = pb.forward(w, "sum")
    outb2 = pb.forward(w, "sum")  # graph replay
    torch.cuda.synchronize()
    check_exact(outb2, outb.cpu().numpy(), "replay")
    # every instance, bit for bit, against the Fenwick pin
    D, Q = _separate_instances(c)
    want = oracle.fenwick2_sums(D, Q, [c.w.astype(np.int64)])[0]
    check_exact(outb, want, "batched vs pin (all 4096 instances)")
    # and against separate plans, one per instance
    ref = torch.empty_like(outb)
    doff, qoff = c.d_offsets, c.q_offsets
    for k in range(len(doff) - 1):
        p = DomAggPlan(d[doff[k]:doff[k + 1]], q[qoff[k]:qoff[k + 1]])
        p.forward(w[doff[k]:doff[k + 1]], "sum", out=ref[qoff[k]:qoff[k + 1]])
        p.close()
    check_exact(outb, ref.cpu().numpy(), "batched vs per-instance")


def test_batched_gmm4d_every_instance():
    """m = 4 batch: on every one of the 64 instances, 256 sampled queries
    (fp32 sum within tolerance, int32 max bit for bit) and 256 sampled
    gradient entries against the fp64 definition; fp32 forward and backward
    replays bit for bit; max equal to a separate plan of the instance."""
    from paper_2305_16751_amd import DomAggPlan
    c = workloads.batched_gmm4d()
    print(f"batched_gmm4d instances={len(c.d_offsets) - 1} points={c.n}", flush=True)
    d, q = to_dev(c.D), to_dev(c.Q)
    w, wi = to_dev(c.w), to_dev(c.w_alt)
    pb = DomAggPlan(d, q, c.d_offsets, c.q_offsets)
    info = pb.info()
    assert info["key_bits"] > 32
    g = np.random.default_rng(6).standard_normal(c.Q.shape[0]).astype(np.float32)
    gd = to_dev(g)
    out = pb.forward(w, "sum").cpu().numpy()
    mx = pb.forward(wi, "max").cpu().numpy()
    gw = pb.backward(gd).cpu().numpy()
    for _ in range(2):
        assert np.array_equal(pb.forward(w, "sum").cpu().numpy(), out), "fp32 forward replay"
        assert np.array_equal(pb.backward(gd).cpu().numpy(), gw), "fp32 backward replay"
    del pb
    _free()
    doff, qoff = c.d_offsets, c.q_offsets
    for k in range(len(doff) - 1):
        D, Q = c.D[doff[k]:doff[k + 1]], c.Q[qoff[k]:qoff[k + 1]]
        wk = c.w[doff[k]:doff[k + 1]].astype(np.float64)
        qi = _sample(Q.shape[0], 256, int(k))
        want = oracle.brute(4, D, Q[qi], wk, "sum")
        scale = oracle.brute(4, D, Q[qi], np.abs(wk), "sum")
        check_fp(torch.from_numpy(out[qoff[k]:qoff[k + 1]][qi]), want, scale, f"sum inst {k}")
        wik = c.w_alt[doff[k]:doff[k + 1]]
        check_exact(torch.from_numpy(mx[qoff[k]:qoff[k + 1]][qi]),
                    oracle.brute(4, D, Q[qi], wik, "max", weight_dtype=np.int32), f"max inst {k}")
        gk = g[qoff[k]:qoff[k + 1]].astype(np.float64)
        dj = _sample(D.shape[0], 256, int(k) + 1)
        gwant = oracle.brute(4, -Q.astype(np.float64), -D[dj].astype(np.float64), gk, "sum")
        gscale = oracle.brute(4, -Q.astype(np.float64), -D[dj].astype(np.float64), np.abs(gk), "sum")
        check_fp(torch.from_numpy(gw[doff[k]:doff[k + 1]][dj]), gwant, gscale, f"grad inst {k}")
    for k in _sample(len(doff) - 1, 4, 7):
        D, Q = c.D[doff[k]:doff[k + 1]], c.Q[qoff[k]:qoff[k + 1]]
        p = DomAggPlan(to_dev(D), to_dev(Q))
        check_exact(p.forward(to_dev(c.w_alt[doff[k]:doff[k + 1]]), "max"), mx[qoff[k]:qoff[k + 1]],
                    f"max per-instance {k}")
        p.close()
