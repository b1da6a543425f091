"""Pins of the CPU oracle against things other than itself.

The oracle's construction (Sec. 4 + Sec. 5) and its plain definition
(Sec. 1.2) are each checked against: the worked examples the paper prints
(golden fixtures), Lemma 1 and Lemma 2 exhaustively for small widths, closed
forms, the textbook special cases (m = 1 prefix aggregation, the m = 2 sweep
with a Fenwick tree), exact size formulas for the flat map, and invariants.
No GPU is needed.
"""
import itertools
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
import workloads


def _read_golden(golden_dir, name):
    rows = {}
    with open(os.path.join(golden_dir, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            rows[k.strip()] = v.split()
    return rows


# --------------------------------------------------------------------------
# Worked examples the paper prints


def test_sscan_worked_example(golden_dir):
    g = _read_golden(golden_dir, "sscan_example.txt")
    a = np.array(g["a"], dtype=float)
    t = np.array(g["t"], dtype=np.int64)
    np.testing.assert_array_equal(oracle.sscan(a, t), np.array(g["out"], dtype=float))


def test_prefix_set_worked_example(golden_dir):
    g = _read_golden(golden_dir, "prefix_set_example.txt")
    x = int(g["x"][0], 2)
    L = len(g["x"][0])
    p0 = {"" if s == "-" else s for s in g["P0"]}
    assert set(oracle.prefix_set(x, L, 0)) == p0
    assert set(oracle.prefix_set(x, L, 1)) == set(g["P1(derived)"])


def test_worked_example_2d(golden_dir):
    g = _read_golden(golden_dir, "worked_example_2d.txt")
    D = np.array([s.split(",") for s in g["D"]], dtype=float)
    Q = np.array([s.split(",") for s in g["Q"]], dtype=float)
    w = np.array(g["w"], dtype=np.int64)
    out, E, L = oracle.construction(2, D, Q, w, "sum", return_stats=True)
    np.testing.assert_array_equal(out, np.array(g["sum"], dtype=np.int64))
    assert E == int(g["E"][0]) and L == [int(g["L"][0])]
    mx = oracle.construction(2, D, Q, w.astype(np.float64), "max")
    np.testing.assert_array_equal(mx, np.array(g["max"], dtype=float))
    np.testing.assert_array_equal(oracle.construction(2, D, Q, None, "count"),
                                  np.array(g["count"], dtype=np.int64))
    np.testing.assert_array_equal(oracle.brute(2, D, Q, w, "sum"), np.array(g["sum"], dtype=np.int64))


# --------------------------------------------------------------------------
# Lemma 1 and Lemma 2, exhaustively for small widths


@pytest.mark.parametrize("L", range(0, 9))
def test_lemma1_exhaustive(L):
    for x in range(1 << L):
        p0 = set(oracle.prefix_set(x, L, 0))
        assert len(p0) == L - bin(x).count("1")
        for y in range(1 << L):
            p1 = set(oracle.prefix_set(y, L, 1))
            assert len(p0 & p1) == (1 if x < y else 0), (L, x, y)


def test_lemma2_tuples():
    L = (3, 2, 3)
    rng = np.random.default_rng(5)
    for _ in range(3000):
        x = [int(rng.integers(0, 1 << l)) for l in L]
        y = [int(rng.integers(0, 1 << l)) for l in L]
        px = list(itertools.product(*[oracle.prefix_set(a, l, 0) for a, l in zip(x, L)]))
        py = set(itertools.product(*[oracle.prefix_set(b, l, 1) for b, l in zip(y, L)]))
        inter = [t for t in px if t in py]
        want = 1 if all(a < b for a, b in zip(x, y)) else 0
        assert len(inter) == want


# --------------------------------------------------------------------------
# Ranks


def test_dense_rank_matches_unique():
    rng = np.random.default_rng(1)
    v = rng.integers(0, 50, size=1000).astype(float)
    v[::7] = -0.0
    v[::11] = 0.0
    r, K = oracle.dense_rank(v)
    u, inv = np.unique(v, return_inverse=True)
    np.testing.assert_array_equal(r, inv)
    assert K == u.size


@pytest.mark.parametrize("K,L", [(0, 0), (1, 0), (2, 1), (3, 2), (4, 2), (5, 3), (1 << 20, 20), ((1 << 20) + 1, 21)])
def test_bits_for(K, L):
    assert oracle.bits_for(K) == L
    if K > 1:
        assert L == math.ceil(math.log2(K))


# --------------------------------------------------------------------------
# Construction vs definition on tiny inputs with heavy ties


def _check_all(m, D, Q, w, op, exact=True):
    a = oracle.construction(m, D, Q, w, op)
    b = oracle.brute(m, D, Q, w, op)
    c = oracle.construction_basic(m, D, Q, w, op)
    if exact:
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(c, b)
    else:
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(c, b, rtol=1e-12, atol=1e-12)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(m=st.integers(1, 4), nD=st.integers(0, 40), nQ=st.integers(0, 40),
       alphabet=st.sampled_from([1, 2, 3, 5, 16]), op=st.sampled_from(["sum", "max", "count"]),
       seed=st.integers(0, 2**31 - 1))
def test_construction_vs_definition_int(m, nD, nQ, alphabet, op, seed):
    c = workloads.small_case(seed, m, nD, nQ, alphabet=alphabet, coord="int", weight="int64")
    _check_all(m, c.D, c.Q, c.w, op)


@settings(max_examples=100, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(m=st.integers(1, 4), nD=st.integers(0, 40), nQ=st.integers(0, 40),
       alphabet=st.sampled_from([2, 4, None]), op=st.sampled_from(["sum", "max"]),
       seed=st.integers(0, 2**31 - 1))
def test_construction_vs_definition_float(m, nD, nQ, alphabet, op, seed):
    c = workloads.small_case(seed, m, nD, nQ, alphabet=alphabet, coord="f32", weight="f64")
    _check_all(m, c.D, c.Q, c.w, op, exact=(op == "max"))


def test_construction_medium_int_3d():
    c = workloads.small_case(7, 3, 600, 500, alphabet=40, coord="int", weight="int64")
    for op in ("sum", "max", "count"):
        _check_all(3, c.D, c.Q, c.w, op)


def test_construction_medium_int_4d():
    c = workloads.small_case(8, 4, 300, 300, alphabet=12, coord="int", weight="int64")
    for op in ("sum", "count"):
        _check_all(4, c.D, c.Q, c.w, op)


def test_signed_zero_and_inf_coordinates():
    D = np.array([[-0.0, 1.0], [0.0, -np.inf], [np.inf, 0.0], [-1.0, -1.0]])
    Q = np.array([[0.0, 2.0], [np.inf, np.inf], [1e-300, 0.5], [-0.0, 3.0]])
    w = np.array([1, 2, 4, 8], dtype=np.int64)
    _check_all(2, D, Q, w, "sum")
    # -0.0 and +0.0 are the same real number: neither dominates the other
    assert oracle.brute(2, D[:1], Q[3:], w[:1], "sum")[0] == 0


def test_nan_rejected():
    D = np.array([[np.nan, 1.0]])
    Q = np.array([[1.0, 2.0]])
    with pytest.raises(oracle.OracleError):
        oracle.construction(2, D, Q, np.array([1], dtype=np.int64))
    with pytest.raises(oracle.OracleError):
        oracle.brute(2, D, Q, np.array([1], dtype=np.int64))


# --------------------------------------------------------------------------
# Closed forms (pins of the plain definition and of the construction)


@pytest.mark.parametrize("m,k", [(1, 9), (2, 7), (3, 5), (4, 4)])
def test_grid_count_closed_form(m, k):
    """D = Q = {0..k-1}^m, w = 1: the count below q is prod(q_i)."""
    g = np.array(list(itertools.product(range(k), repeat=m)), dtype=float)
    want = np.prod(g, axis=1).astype(np.int64)
    np.testing.assert_array_equal(oracle.construction(m, g, g, None, "count"), want)
    np.testing.assert_array_equal(oracle.brute(m, g, g, None, "count"), want)


def test_separable_weights_closed_form():
    """w(d) = prod f_i(d_i) on a full grid: sum(q) = prod_i sum_{x<q_i} f_i(x)."""
    k, m = 6, 3
    rng = np.random.default_rng(3)
    f = rng.integers(-5, 6, size=(m, k)).astype(np.int64)
    g = np.array(list(itertools.product(range(k), repeat=m)), dtype=np.int64)
    w = np.prod(np.stack([f[i][g[:, i]] for i in range(m)]), axis=0)
    pre = np.concatenate([np.zeros((m, 1), np.int64), np.cumsum(f, axis=1)], axis=1)
    want = np.prod(np.stack([pre[i][g[:, i]] for i in range(m)]), axis=0)
    np.testing.assert_array_equal(oracle.construction(m, g.astype(float), g.astype(float), w, "sum"), want)
    np.testing.assert_array_equal(oracle.brute(m, g.astype(float), g.astype(float), w, "sum"), want)


def test_antichain_all_identity():
    """Points on x1 + x2 = const: no point dominates another."""
    x = np.arange(50, dtype=float)
    P = np.stack([x, 49 - x], axis=1)
    w = np.arange(50, dtype=np.int64) + 1
    np.testing.assert_array_equal(oracle.construction(2, P, P, w, "sum"), np.zeros(50, np.int64))
    mx = oracle.construction(2, P, P, w, "max")
    assert (mx == np.iinfo(np.int64).min).all()


def test_m1_is_prefix_aggregation():
    """m = 1: sort D, prefix-sum, strict lower bound per query (Sec. 1.1)."""
    rng = np.random.default_rng(11)
    D = rng.integers(0, 300, size=2000).astype(float)
    Q = rng.integers(0, 300, size=1500).astype(float)
    w = rng.integers(0, 1000, size=2000).astype(np.int64)
    order = np.argsort(D, kind="stable")
    pre = np.concatenate([[0], np.cumsum(w[order])])
    want = pre[np.searchsorted(D[order], Q, side="left")]
    np.testing.assert_array_equal(oracle.construction(1, D[:, None], Q[:, None], w, "sum"), want)
    np.testing.assert_array_equal(oracle.brute(1, D[:, None], Q[:, None], w, "sum"), want)


# --------------------------------------------------------------------------
# The m = 2 textbook sweep (a different algorithm) at medium size


def test_fenwick_pins_construction_int():
    c = workloads.int2d_64k(n=1 << 13)
    for op in ("sum", "max", "count"):
        np.testing.assert_array_equal(oracle.construction(2, c.D, c.Q, c.w, op),
                                      oracle.fenwick2(c.D, c.Q, c.w, op))


def test_fenwick_pins_definition_small():
    c = workloads.small_case(21, 2, 300, 300, alphabet=20)
    for op in ("sum", "max", "count"):
        np.testing.assert_array_equal(oracle.brute(2, c.D, c.Q, c.w, op), oracle.fenwick2(c.D, c.Q, c.w, op))


def test_fenwick_pins_construction_float():
    c = workloads.f32_uniform(2, 1 << 12, 99, "t")
    w = c.w.astype(np.float64)
    np.testing.assert_allclose(oracle.construction(2, c.D, c.Q, w, "sum"),
                               oracle.fenwick2(c.D, c.Q, w, "sum"), rtol=1e-12, atol=1e-9)
    np.testing.assert_array_equal(oracle.construction(2, c.D, c.Q, w, "max"),
                                  oracle.fenwick2(c.D, c.Q, w, "max"))


# --------------------------------------------------------------------------
# Size of the flat map (Sec. 5): exact count and the n * prod(L_i) bound


def _expected_E(m, D, Q):
    P = np.concatenate([D, Q]).astype(np.float64)
    nD = D.shape[0]
    cnt = np.ones(P.shape[0], dtype=np.int64)
    Ls = []
    for i in range(m - 1):
        u, r = np.unique(P[:, i], return_inverse=True)
        L = int(math.ceil(math.log2(u.size))) if u.size > 1 else 0
        Ls.append(L)
        pc = np.array([bin(int(x)).count("1") for x in r], dtype=np.int64)
        cnt *= np.where(np.arange(P.shape[0]) < nD, L - pc, pc)
    return int(cnt.sum()), Ls


@pytest.mark.parametrize("m,n,alpha", [(1, 100, 5), (2, 500, 1000), (2, 700, 3), (3, 300, 50), (4, 120, 9)])
def test_expansion_size_formula(m, n, alpha):
    c = workloads.small_case(m * 1000 + n, m, n, n + 7, alphabet=alpha)
    _, E, L = oracle.construction(m, c.D, c.Q, c.w, "sum", return_stats=True)
    E_want, L_want = _expected_E(m, c.D, c.Q)
    assert E == E_want and L == L_want
    assert E <= c.n * int(np.prod(L_want)) if m > 1 else E == c.n


# --------------------------------------------------------------------------
# Invariants


def test_total_count_is_number_of_dominated_pairs():
    c = workloads.small_case(31, 3, 400, 350, alphabet=10)
    cnt = oracle.construction(3, c.D, c.Q, None, "count")
    pairs = int(np.all(c.D[:, None, :] < c.Q[None, :, :], axis=2).sum())
    assert int(cnt.sum()) == pairs


def test_permutation_invariance():
    c = workloads.small_case(41, 3, 300, 250, alphabet=12)
    base = oracle.construction(3, c.D, c.Q, c.w, "sum")
    rng = np.random.default_rng(0)
    pd = rng.permutation(c.D.shape[0])
    pq = rng.permutation(c.Q.shape[0])
    out = oracle.construction(3, c.D[pd], c.Q[pq], c.w[pd], "sum")
    np.testing.assert_array_equal(out, base[pq])


def test_monotone_map_invariance():
    c = workloads.small_case(51, 2, 400, 400, alphabet=30)
    base = oracle.construction(2, c.D, c.Q, c.w, "sum")
    f = lambda x: np.exp(0.3 * x) - 7.0  # strictly increasing
    out = oracle.construction(2, f(c.D.astype(float)), f(c.Q.astype(float)), c.w, "sum")
    np.testing.assert_array_equal(out, base)


def test_transposed_sum_is_gradient():
    """The loss sum_q c_q out_q is linear in w; its gradient is the transposed
    dominance sum.  Checked by the definition and by exact finite differences."""
    c = workloads.small_case(61, 2, 120, 110, alphabet=9, weight="f64")
    g = np.random.default_rng(2).standard_normal(c.Q.shape[0])
    grad = oracle.transposed_sum(2, c.D, c.Q, g)
    dom = np.all(c.D[:, None, :] < c.Q[None, :, :], axis=2)
    np.testing.assert_allclose(grad, dom.astype(float) @ g, rtol=1e-12, atol=1e-12)
    eps = 1e-3
    for i in range(0, c.D.shape[0], 17):
        wp, wm = c.w.copy(), c.w.copy()
        wp[i] += eps
        wm[i] -= eps
        fd = (g @ oracle.construction(2, c.D, c.Q, wp, "sum") - g @ oracle.construction(2, c.D, c.Q, wm, "sum")) / (2 * eps)
        assert abs(fd - grad[i]) < 1e-8 * (1 + abs(grad[i]))


def test_empty_inputs():
    D = np.zeros((0, 2))
    Q = np.array([[1.0, 1.0]])
    assert oracle.construction(2, D, Q, np.zeros(0, np.int64), "sum").tolist() == [0]
    assert oracle.construction(2, Q, D, np.ones(1, np.int64), "sum").size == 0
    out, E, L = oracle.construction(3, np.ones((5, 3)), np.ones((4, 3)), np.ones(5, np.int64), "sum",
                                    return_stats=True)
    assert E == 0 and L == [0, 0] and out.tolist() == [0] * 4
