"""The HIP path's variants against the oracle, element by element:
non-strict dominance (DOM_AGG_LE: <= on chosen axes, e.g. the multivariate
empirical CDF) and the basic construction of Sec. 4 (DOM_AGG_BASIC: every
axis expanded, data before queries on ties), through the C-ABI.  Integer F
and max bit-exact; fp32 sums within 2e-6 * (sum of |w| over the dominated
set) against fp64.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_helpers import DEV, check_exact, check_fp, to_dev

pytestmark = pytest.mark.gpu


def _plan(c, **kw):
    from paper_2305_16751_amd import DomAggPlan
    return DomAggPlan(to_dev(c.D), to_dev(c.Q), **kw)


def _masks(m):
    return sorted({0, (1 << m) - 1, 1, 1 << (m - 1)} | ({5} if m >= 3 else set()))


SIZES = {1: 3000, 2: 2500, 3: 900, 4: 300}


@pytest.mark.parametrize("m", [1, 2, 3, 4])
@pytest.mark.parametrize("coord,alpha", [("int", 6), ("int", 1 << 20), ("f32", 16)])
def test_le_int_weights(m, coord, alpha):
    n = SIZES[m]
    for le in _masks(m):
        c = workloads.small_case(700 + 13 * m + le + (alpha % 97), m, n, n - 29, alphabet=alpha, coord=coord,
                                 weight="int64")
        print(f"le m={m} {coord} alpha={alpha} le_mask={le}", flush=True)
        p = _plan(c, le_mask=le)
        want, E, L = oracle.construction(m, c.D, c.Q, c.w, "sum", return_stats=True, le_mask=le)
        info = p.info()
        assert info["records"] == E and info["L"] == L and info["le_mask"] == le, (info, E, L)
        check_exact(p.forward(to_dev(c.w), "sum"), want, f"sum le={le}")
        check_exact(p.forward(to_dev(c.w), "max"), oracle.construction(m, c.D, c.Q, c.w, "max", le_mask=le),
                    f"max le={le}")
        check_exact(p.forward(None, "count"), oracle.construction(m, c.D, c.Q, None, "count", le_mask=le),
                    f"count le={le}")


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_le_float_weights_and_gradient(m):
    n = SIZES[m]
    for le in _masks(m):
        c = workloads.small_case(800 + 7 * m + le, m, n - 3, n, alphabet=12, coord="f32", weight="f32")
        print(f"le float m={m} le_mask={le}", flush=True)
        p = _plan(c, le_mask=le)
        w64 = c.w.astype(np.float64)
        check_fp(p.forward(to_dev(c.w), "sum"), oracle.construction(m, c.D, c.Q, w64, "sum", le_mask=le),
                 oracle.construction(m, c.D, c.Q, np.abs(w64), "sum", le_mask=le), f"sum f32 le={le}")
        g = np.random.default_rng(m + le).standard_normal(c.Q.shape[0]).astype(np.float32)
        g64 = g.astype(np.float64)
        check_fp(p.backward(to_dev(g)), oracle.transposed_sum(m, c.D, c.Q, g64, le_mask=le),
                 oracle.transposed_sum(m, c.D, c.Q, np.abs(g64), le_mask=le), f"grad le={le}")


@pytest.mark.parametrize("m", [2, 3])
def test_le_one_shot_and_batched(m):
    from paper_2305_16751_amd import dom_agg_run
    le = (1 << m) - 1
    c = workloads.small_case(900 + m, m, 2000, 1900, alphabet=40, coord="int", weight="int64")
    w32 = c.w.astype(np.int32)
    got = dom_agg_run(to_dev(c.D), to_dev(c.Q), to_dev(w32), "sum", le_mask=le)
    check_exact(got, oracle.construction(m, c.D, c.Q, w32.astype(np.int64), "sum", le_mask=le), "one-shot le")
    # two instances stacked
    doff = np.array([0, 700, 2000], dtype=np.int64)
    qoff = np.array([0, 1000, 1900], dtype=np.int64)
    from paper_2305_16751_amd import DomAggPlan
    pb = DomAggPlan(to_dev(c.D), to_dev(c.Q), doff, qoff, le_mask=le)
    out = pb.forward(to_dev(c.w), "sum").cpu().numpy()
    for k in range(2):
        want = oracle.construction(m, c.D[doff[k]:doff[k + 1]], c.Q[qoff[k]:qoff[k + 1]], c.w[doff[k]:doff[k + 1]],
                                   "sum", le_mask=le)
        check_exact(torch.from_numpy(out[qoff[k]:qoff[k + 1]]), want, f"batched le instance {k}")


def test_ecdf_2d_1m_every_count():
    """The multivariate empirical CDF of 2^20 float32 points at 2^20 query
    points (<= on both axes), every count exact against the textbook sweep."""
    c = workloads.f32_uniform(2, 1 << 20, workloads.BASE_SEED + 31, "ecdf")
    print("ecdf 2d 1M", flush=True)
    p = _plan(c, le_mask=3)
    cnt = p.forward(None, "count").cpu().numpy()
    np.testing.assert_array_equal(cnt, oracle.sweep(2, c.D, c.Q, None, "count", le_mask=3))


# ---------------------------------------------------------------------------
# the basic variant


@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("coord,alpha", [("int", 6), ("int", 1 << 20), ("f32", 16), ("f32", None)])
def test_basic_matches_oracle_and_sec5(m, coord, alpha):
    n = {1: 3000, 2: 1500, 3: 500}[m]
    c = workloads.small_case(1000 + 11 * m + (alpha or 0) % 89, m, n, n - 17, alphabet=alpha, coord=coord,
                             weight="int64")
    print(f"basic m={m} {coord} alpha={alpha}", flush=True)
    p = _plan(c, basic=True)
    want, E, L = oracle.construction_basic(m, c.D, c.Q, c.w, "sum", return_stats=True)
    info = p.info()
    assert info["basic"] == 1 and info["records"] == E and info["L"] == L, (info, E, L)
    got = p.forward(to_dev(c.w), "sum")
    check_exact(got, want, "basic sum")
    check_exact(got, _plan(c).forward(to_dev(c.w), "sum").cpu().numpy(), "basic vs Sec. 5")
    check_exact(p.forward(to_dev(c.w), "max"), oracle.construction_basic(m, c.D, c.Q, c.w, "max"), "basic max")
    check_exact(p.forward(None, "count"), oracle.construction_basic(m, c.D, c.Q, None, "count"), "basic count")
    wf = (c.w.astype(np.float64) * 0.01).astype(np.float32)
    w64 = wf.astype(np.float64)
    check_fp(p.forward(to_dev(wf), "sum"), oracle.construction_basic(m, c.D, c.Q, w64, "sum"),
             oracle.construction_basic(m, c.D, c.Q, np.abs(w64), "sum"), "basic f32 sum")
    g = np.random.default_rng(m).standard_normal(c.Q.shape[0]).astype(np.float32)
    g64 = g.astype(np.float64)
    check_fp(p.backward(to_dev(g)), oracle.transposed_sum(m, c.D, c.Q, g64),
             oracle.transposed_sum(m, c.D, c.Q, np.abs(g64)), "basic grad")


@pytest.mark.parametrize("m", [2, 3])
def test_basic_le_one_shot_and_batch(m):
    from paper_2305_16751_amd import DomAggPlan, dom_agg_run
    c = workloads.small_case(1100 + m, m, 1200, 1100, alphabet=30, coord="int", weight="int64")
    le = 1 << (m - 1)
    p = _plan(c, basic=True, le_mask=le)
    want, E = oracle.construction_basic(m, c.D, c.Q, c.w, "sum", return_E=True, le_mask=le)
    assert p.info()["records"] == E
    check_exact(p.forward(to_dev(c.w), "sum"), want, "basic le")
    w32 = c.w.astype(np.int32)
    check_exact(dom_agg_run(to_dev(c.D), to_dev(c.Q), to_dev(w32), "sum", basic=True, le_mask=le),
                oracle.construction_basic(m, c.D, c.Q, w32.astype(np.int64), "sum", le_mask=le), "basic one-shot")
    doff = np.array([0, 0, 500, 1200], dtype=np.int64)
    qoff = np.array([0, 300, 300, 1100], dtype=np.int64)
    pb = DomAggPlan(to_dev(c.D), to_dev(c.Q), doff, qoff, basic=True)
    out = pb.forward(to_dev(c.w), "sum").cpu().numpy()
    for k in range(3):
        if qoff[k + 1] > qoff[k]:
            want = oracle.construction_basic(m, c.D[doff[k]:doff[k + 1]], c.Q[qoff[k]:qoff[k + 1]],
                                             c.w[doff[k]:doff[k + 1]], "sum")
            check_exact(torch.from_numpy(out[qoff[k]:qoff[k + 1]]), want, f"basic batched instance {k}")


def test_basic_rejects_m4():
    from paper_2305_16751_amd import DomAggError, DomAggPlan
    x = torch.rand((10, 4), device=DEV)
    with pytest.raises(DomAggError, match="EUNSUPPORTED"):
        DomAggPlan(x, x, basic=True)
