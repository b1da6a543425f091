"""The HIP path at the full workload sizes, in the launch configuration the
benchmark times (default plan, autotuned tiles), against the oracle.

Where the oracle's construction would take minutes at full size, sampled
outputs are checked against the plain definition computed one by one
(oracle.brute on the sampled queries; oracle.brute on swapped, negated roles
for sampled gradient entries), plus properties at full size (the exact count
of a textbook sweep for m = 2).
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


def test_f32_2d_2m_counts_and_sums():
    """Medium size between the small cases and the full workload: long
    segments (look-back chains over hundreds of tiles), every count exact."""
    c = workloads.f32_uniform(2, 1 << 21, workloads.BASE_SEED + 21, "f32_2d_2m")
    print(f"f32_2d_2m |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    p = _plan(c.D, c.Q)
    cnt = p.forward(None, "count").cpu().numpy()
    np.testing.assert_array_equal(cnt, oracle.fenwick2(c.D, c.Q, None, "count"))
    out = p.forward(to_dev(c.w), "sum").cpu().numpy()
    idx = _sample(c.Q.shape[0], 256, 9)
    w64 = c.w.astype(np.float64)
    check_fp(torch.from_numpy(out[idx]), oracle.brute(2, c.D, c.Q[idx], w64, "sum"),
             oracle.brute(2, c.D, c.Q[idx], np.abs(w64), "sum"), "f32_2d_2m sum")
    g = np.random.default_rng(10).standard_normal(c.Q.shape[0]).astype(np.float32)
    gw = p.backward(to_dev(g)).cpu().numpy()
    di = _sample(c.D.shape[0], 256, 11)
    g64 = g.astype(np.float64)
    check_fp(torch.from_numpy(gw[di]), oracle.brute(2, -c.Q.astype(np.float64), -c.D[di].astype(np.float64), g64, "sum"),
             oracle.brute(2, -c.Q.astype(np.float64), -c.D[di].astype(np.float64), np.abs(g64), "sum"), "grad")


def test_f32_2d_16m_sampled():
    c = workloads.f32_2d_16m()
    print(f"f32_2d_16m |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    p = _plan(c.D, c.Q)
    out = p.forward(to_dev(c.w), "sum").cpu().numpy()
    cnt = p.forward(None, "count").cpu().numpy()
    info = p.info()
    del p
    torch.cuda.empty_cache()
    # every count, exactly, by the textbook sweep (a property at full size)
    np.testing.assert_array_equal(cnt, oracle.fenwick2(c.D, c.Q, None, "count"))
    # sampled sums against the definition in fp64
    idx = _sample(c.Q.shape[0], 96, 1)
    w64 = c.w.astype(np.float64)
    want = oracle.brute(2, c.D, c.Q[idx], w64, "sum")
    scale = oracle.brute(2, c.D, c.Q[idx], np.abs(w64), "sum")
    check_fp(torch.from_numpy(out[idx]), want, scale, "f32_2d_16m sum")
    assert info["records"] > 0


def test_f32_3d_1m_sampled():
    c = workloads.f32_3d_1m()
    print(f"f32_3d_1m |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    p = _plan(c.D, c.Q)
    out = p.forward(to_dev(c.w), "sum").cpu().numpy()
    cnt = p.forward(None, "count").cpu().numpy()
    idx = _sample(c.Q.shape[0], 256, 2)
    w64 = c.w.astype(np.float64)
    want = oracle.brute(3, c.D, c.Q[idx], w64, "sum")
    scale = oracle.brute(3, c.D, c.Q[idx], np.abs(w64), "sum")
    check_fp(torch.from_numpy(out[idx]), want, scale, "f32_3d_1m sum")
    np.testing.assert_array_equal(cnt[idx], oracle.brute(3, c.D, c.Q[idx], None, "count"))


def test_f32_2d_4m_grad():
    """Forward + adjoint; gradient vs the fp64 definition on sampled data
    points and vs central finite differences of the fp64 loss."""
    from paper_2305_16751_amd import dom_agg, DomAggPlan
    c = workloads.f32_2d_4m_grad()
    print(f"f32_2d_4m_grad |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    d, q = to_dev(c.D), to_dev(c.Q)
    w = to_dev(c.w).requires_grad_(True)
    out = dom_agg(d, q, w, "sum")
    loss = (out * to_dev(c.c)).sum()
    loss.backward()
    grad = w.grad.cpu().numpy().astype(np.float64)
    di = _sample(c.D.shape[0], 512, 3)
    c64 = c.c.astype(np.float64)
    # grad[i] = sum of c_q over q with D[i] < q  ==  brute(-Q as data with weights c, -D[i] as queries)
    want = oracle.brute(2, -c.Q.astype(np.float64), -c.D[di].astype(np.float64), c64, "sum")
    scale = oracle.brute(2, -c.Q.astype(np.float64), -c.D[di].astype(np.float64), np.abs(c64), "sum")
    check_fp(torch.from_numpy(grad[di]), want, scale, "grad vs definition")
    # finite differences of the fp64 loss (the GPU path with float64 weights)
    plan = DomAggPlan(d, q)
    w64 = to_dev(c.w.astype(np.float64))
    cq = to_dev(c64)
    rng = np.random.default_rng(4)
    v = np.zeros(c.D.shape[0])
    v[di] = rng.standard_normal(di.size)
    vd = to_dev(v)
    eps = 1e-3
    lp = float((plan.forward(w64 + eps * vd, "sum") * cq).sum())
    lm = float((plan.forward(w64 - eps * vd, "sum") * cq).sum())
    fd = (lp - lm) / (2 * eps)
    gv = float(grad @ v)
    assert abs(fd - gv) <= 1e-4 * (abs(gv) + np.abs(grad[di]) @ np.abs(v[di])), (fd, gv)
    for i in di[:16]:
        e = torch.zeros(c.D.shape[0], dtype=torch.float64, device=DEV)
        e[int(i)] = eps
        fdi = (float((plan.forward(w64 + e, "sum") * cq).sum()) - float((plan.forward(w64 - e, "sum") * cq).sum())) / (2 * eps)
        assert abs(fdi - grad[i]) <= 1e-4 * (abs(grad[i]) + 1.0), (int(i), fdi, grad[i])


def test_batched_int2d_matches_per_instance():
    from paper_2305_16751_amd import DomAggPlan
    c = workloads.batched_int2d()
    print(f"batched_int2d instances={len(c.d_offsets) - 1} points={c.n}", flush=True)
    d, q, w = to_dev(c.D), to_dev(c.Q), to_dev(c.w)
    pb = DomAggPlan(d, q, c.d_offsets, c.q_offsets, graph=True)
    outb = pb.forward(w, "sum")
    outb2 = pb.forward(w, "sum")  # graph replay
    torch.cuda.synchronize()
    check_exact(outb2, outb.cpu().numpy(), "replay")
    ref = torch.empty_like(outb)
    doff, qoff = c.d_offsets, c.q_offsets
    for k in range(len(doff) - 1):
        p = DomAggPlan(d[doff[k]:doff[k + 1]], q[qoff[k]:qoff[k + 1]])
        p.forward(w[doff[k]:doff[k + 1]], "sum", out=ref[qoff[k]:qoff[k + 1]])
        p.close()
    check_exact(outb, ref.cpu().numpy(), "batched vs per-instance")
    ob = outb.cpu().numpy()
    for k in _sample(len(doff) - 1, 6, 5):
        D, Q = c.D[doff[k]:doff[k + 1]], c.Q[qoff[k]:qoff[k + 1]]
        check_exact(torch.from_numpy(ob[qoff[k]:qoff[k + 1]]),
                    oracle.construction(2, D, Q, c.w[doff[k]:doff[k + 1]], "sum"), f"instance {k}")


def test_batched_gmm4d():
    """m = 4 batch: fp32 sum forward + backward vs per-instance plans and the
    definition on sampled points; int32 max bit-exact on sampled queries."""
    from paper_2305_16751_amd import DomAggPlan
    c = workloads.batched_gmm4d()
    print(f"batched_gmm4d instances={len(c.d_offsets) - 1} points={c.n}", flush=True)
    d, q = to_dev(c.D), to_dev(c.Q)
    w, wi = to_dev(c.w), to_dev(c.w_alt)
    pb = DomAggPlan(d, q, c.d_offsets, c.q_offsets)
    info = pb.info()
    assert info["key_bits"] > 32
    out = pb.forward(w, "sum").cpu().numpy()
    mx = pb.forward(wi, "max").cpu().numpy()
    g = np.random.default_rng(6).standard_normal(c.Q.shape[0]).astype(np.float32)
    gw = pb.backward(to_dev(g)).cpu().numpy()
    del pb
    torch.cuda.empty_cache()
    doff, qoff = c.d_offsets, c.q_offsets
    for k in _sample(len(doff) - 1, 5, 7):
        D, Q = c.D[doff[k]:doff[k + 1]], c.Q[qoff[k]:qoff[k + 1]]
        wk = c.w[doff[k]:doff[k + 1]].astype(np.float64)
        qi = _sample(Q.shape[0], 64, int(k))
        want = oracle.brute(4, D, Q[qi], wk, "sum")
        scale = oracle.brute(4, D, Q[qi], np.abs(wk), "sum")
        check_fp(torch.from_numpy(out[qoff[k]:qoff[k + 1]][qi]), want, scale, f"sum inst {k}")
        wik = c.w_alt[doff[k]:doff[k + 1]]
        check_exact(torch.from_numpy(mx[qoff[k]:qoff[k + 1]][qi]),
                    oracle.brute(4, D, Q[qi], wik, "max", weight_dtype=np.int32), f"max inst {k}")
        gk = g[qoff[k]:qoff[k + 1]].astype(np.float64)
        dj = _sample(D.shape[0], 64, int(k) + 1)
        gwant = oracle.brute(4, -Q.astype(np.float64), -D[dj].astype(np.float64), gk, "sum")
        gscale = oracle.brute(4, -Q.astype(np.float64), -D[dj].astype(np.float64), np.abs(gk), "sum")
        check_fp(torch.from_numpy(gw[doff[k]:doff[k + 1]][dj]), gwant, gscale, f"grad inst {k}")
        # the same instance on its own plan
        p = DomAggPlan(to_dev(D), to_dev(Q))
        check_exact(p.forward(to_dev(wik), "max"), mx[qoff[k]:qoff[k + 1]], f"max per-instance {k}")
        p.close()


def test_f32_2d_16m_one_shot():
    """The one-shot entry point at the full size: every count exact (Fenwick
    sweep), sampled sums against the fp64 definition."""
    from paper_2305_16751_amd import dom_agg_run
    c = workloads.f32_2d_16m()
    print(f"f32_2d_16m one-shot |D|={c.D.shape[0]} |Q|={c.Q.shape[0]}", flush=True)
    d, q = to_dev(c.D), to_dev(c.Q)
    out = dom_agg_run(d, q, to_dev(c.w), "sum").cpu().numpy()
    cnt = dom_agg_run(d, q, None, "count").cpu().numpy()
    del d, q
    torch.cuda.empty_cache()
    np.testing.assert_array_equal(cnt, oracle.fenwick2(c.D, c.Q, None, "count"))
    idx = _sample(c.Q.shape[0], 96, 12)
    w64 = c.w.astype(np.float64)
    check_fp(torch.from_numpy(out[idx]), oracle.brute(2, c.D, c.Q[idx], w64, "sum"),
             oracle.brute(2, c.D, c.Q[idx], np.abs(w64), "sum"), "f32_2d_16m one-shot sum")
