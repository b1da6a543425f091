"""Pins of the oracle's extensions: non-strict dominance (<= on chosen axes,
the ECDF use of Sec. 1.2), the final list of Sec. 4 (its last instructions,
6m+6 .. 6m+9, and the shortcut for monotone F), the basic variant with
<=, and the textbook divide-and-conquer sweep used to pin the GPU path at
full size.  Each is checked against something other than itself: the
definition by brute force, closed forms, textbook special cases, and an
independent pair formula for the data entries of the final list.  No GPU.
"""
import itertools

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
import workloads


def _case(seed, m, nD, nQ, alpha, weight="int64", coord="int"):
    return workloads.small_case(seed, m, nD, nQ, alphabet=alpha, coord=coord, weight=weight)


# --------------------------------------------------------------------------
# non-strict dominance


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_le_construction_equals_definition_every_mask(m):
    for le in range(1 << m):
        c = _case(40 + 3 * m + le, m, 120 if m < 4 else 60, 100 if m < 4 else 50, 5)
        for op in ("sum", "max", "count"):
            w = None if op == "count" else c.w
            want = oracle.brute(m, c.D, c.Q, w, op, le_mask=le)
            np.testing.assert_array_equal(oracle.construction(m, c.D, c.Q, w, op, le_mask=le), want)
            np.testing.assert_array_equal(oracle.construction_basic(m, c.D, c.Q, w, op, le_mask=le), want)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(m=st.integers(1, 3), le=st.integers(0, 7), seed=st.integers(0, 10 ** 6), alpha=st.sampled_from([2, 3, 7, 50]),
       nD=st.integers(0, 40), nQ=st.integers(0, 40))
def test_le_random_float_weights(m, le, seed, alpha, nD, nQ):
    le &= (1 << m) - 1
    c = _case(seed, m, nD, nQ, alpha, weight="f64", coord="f32")
    want = oracle.brute(m, c.D, c.Q, c.w, "sum", le_mask=le)
    np.testing.assert_allclose(oracle.construction(m, c.D, c.Q, c.w, "sum", le_mask=le), want, rtol=1e-12,
                               atol=1e-12)
    np.testing.assert_array_equal(oracle.construction(m, c.D, c.Q, c.w, "max", le_mask=le),
                                  oracle.brute(m, c.D, c.Q, c.w, "max", le_mask=le))


@pytest.mark.parametrize("m,k", [(1, 9), (2, 7), (3, 5), (4, 3)])
def test_ecdf_grid_closed_form(m, k):
    """D = Q = the grid {0..k-1}^m, unit weights: a query q counts
    prod (q_a + 1) over <= axes times prod q_a over < axes."""
    grid = np.array(list(itertools.product(range(k), repeat=m)), dtype=np.int32)
    for le in range(1 << m):
        want = np.ones(grid.shape[0], dtype=np.int64)
        for a in range(m):
            want *= grid[:, a].astype(np.int64) + ((le >> a) & 1)
        np.testing.assert_array_equal(oracle.construction(m, grid, grid, None, "count", le_mask=le), want)


def test_m1_le_is_searchsorted_right():
    """m = 1 with <=: the ECDF of D at each query, numpy's right bisection."""
    rng = np.random.default_rng(3)
    D = rng.integers(0, 40, size=(500, 1)).astype(np.int32)
    Q = rng.integers(-2, 42, size=(300, 1)).astype(np.int32)
    want = np.searchsorted(np.sort(D[:, 0]), Q[:, 0], side="right")
    np.testing.assert_array_equal(oracle.construction(1, D, Q, None, "count", le_mask=1), want)
    wantl = np.searchsorted(np.sort(D[:, 0]), Q[:, 0], side="left")
    np.testing.assert_array_equal(oracle.construction(1, D, Q, None, "count", le_mask=0), wantl)


@pytest.mark.parametrize("m", [2, 3])
def test_le_transposed_sum(m):
    c = _case(77 + m, m, 150, 130, 4, weight="f64")
    g = np.random.default_rng(m).standard_normal(c.Q.shape[0])
    for le in range(1 << m):
        want = oracle.brute(m, -c.Q.astype(np.float64), -c.D.astype(np.float64), g, "sum", le_mask=le)
        np.testing.assert_allclose(oracle.transposed_sum(m, c.D, c.Q, g, le_mask=le), want, rtol=1e-12, atol=1e-12)


def test_le_bits_grow_by_one_exactly_at_powers_of_two():
    """With <= the query ranks reach K, so the width is ceil(log2(K + 1)):
    K = 4 distinct values need 2 bits strictly and 3 with <=."""
    D = np.array([[0, 0], [1, 1], [2, 2], [3, 3]], dtype=np.int32)
    _, E0, L0 = oracle.construction(2, D, D, None, "count", return_stats=True)
    _, E1, L1 = oracle.construction(2, D, D, None, "count", return_stats=True, le_mask=1)
    assert L0 == [2] and L1 == [3]


# --------------------------------------------------------------------------
# the divide-and-conquer sweep (a pin of the GPU path at full size)


@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("op", ["sum", "max", "count"])
def test_sweep_equals_definition(m, op):
    for le in range(1 << m):
        for alpha, coord, weight in ((4, "int", "int64"), (None, "f32", "f64"), (16, "f32", "f64")):
            c = _case(900 + m + le + (alpha or 0), m, 333, 271, alpha, weight=weight, coord=coord)
            w = None if op == "count" else c.w
            got = oracle.sweep(m, c.D, c.Q, w, op, le_mask=le)
            want = oracle.brute(m, c.D, c.Q, w, op, le_mask=le)
            if op == "sum" and c.w.dtype.kind == "f":
                np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
            else:
                np.testing.assert_array_equal(got, want)


def test_sweep_equals_fenwick_m2_medium():
    c = workloads.f32_uniform(2, 1 << 15, 5, "m")
    w = c.w.astype(np.float64)
    np.testing.assert_allclose(oracle.sweep(2, c.D, c.Q, w, "sum"), oracle.fenwick2(c.D, c.Q, w, "sum"),
                               rtol=1e-9, atol=1e-9)
    np.testing.assert_array_equal(oracle.sweep(2, c.D, c.Q, None, "count"), oracle.fenwick2(c.D, c.Q, None, "count"))


def test_sweep_signed_zero_and_empty_sides():
    D = np.array([[-0.0, 1.0, 2.0], [0.0, 0.0, 0.0]])
    Q = np.array([[0.0, 1.0, 2.0], [1.0, 2.0, 3.0]])
    np.testing.assert_array_equal(oracle.sweep(3, D, Q, None, "count"), oracle.brute(3, D, Q, None, "count"))
    np.testing.assert_array_equal(oracle.sweep(3, D, Q, None, "count", le_mask=7),
                                  oracle.brute(3, D, Q, None, "count", le_mask=7))
    assert oracle.sweep(3, D[:0], Q, None, "count").tolist() == [0, 0]
    assert oracle.sweep(3, D, Q[:0], None, "count").size == 0


# --------------------------------------------------------------------------
# the final list of Sec. 4


def _ranks_for_list(m, D, Q, le, sec5=True):
    """Per point (ID order) its ranks on the expanded axes as the construction
    uses them (queries +1 on <= axes) and the widths."""
    nD = D.shape[0]
    nt = m - 1 if sec5 else m
    R, L = [], []
    for a in range(nt):
        r, K = oracle.dense_rank(np.concatenate([D[:, a], Q[:, a]]).astype(np.float64))
        r = r.copy()
        if (le >> a) & 1:
            r[nD:] += 1
            K += 1
        R.append(r)
        L.append(oracle.bits_for(K))
    return R, L


def _record_counts(R, L, nD, n):
    cnt = np.ones(n, dtype=np.int64)
    for r, l in zip(R, L):
        pc = np.array([bin(int(x)).count("1") for x in r], dtype=np.int64)
        cnt *= np.where(np.arange(n) < nD, l - pc, pc)
    return cnt


def _data_totals_by_pairs(m, D, w, R, L, le, op, nD):
    """Independent formula for the data entries: at a data record of tuple t
    the scan holds F over the data records of t up to it (Sec. 5 order:
    last coordinate, then ID among data); so a data point's total is F over
    data points d' no later than it on the last axis, each taken once per
    tuple in P0(d) and P0(d') (for a sum: weighted by that number).  Per
    axis, the common elements of P0(x) and P0(y) are the 0-digits of x
    inside the longest common prefix of x and y."""
    out = []
    for i in range(nD):
        acc = None
        for j in range(nD):
            xi, xj = D[i, m - 1], D[j, m - 1]
            if not (xj < xi or (xj == xi and j <= i)):
                continue
            common = 1
            for a in range(m - 1):
                x, y, l = int(R[a][i]), int(R[a][j]), L[a]
                k = 0
                while k < l and ((x >> (l - 1 - k)) & 1) == ((y >> (l - 1 - k)) & 1):
                    k += 1
                common *= sum(1 for t in range(k) if not (x >> (l - 1 - t)) & 1)
            if common == 0:
                continue
            if op == "sum":
                acc = (acc or 0) + common * int(w[j])
            else:
                acc = int(w[j]) if acc is None else max(acc, int(w[j]))
        out.append(acc)
    return out


@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("op", ["sum", "max", "count"])
def test_final_list_against_definition(m, op):
    for le in (0, (1 << m) - 1, 1):
        c = _case(1200 + 5 * m + le, m, 45, 40, 6)
        w = None if op == "count" else c.w
        nD, n = c.D.shape[0], c.D.shape[0] + c.Q.shape[0]
        ids, vals = oracle.final_list(m, c.D, c.Q, w, op, le_mask=le)
        _, E, _ = oracle.construction(m, c.D, c.Q, w, op, return_stats=True, le_mask=le)
        assert ids.size == E and np.all(np.diff(ids) >= 0)
        R, L = _ranks_for_list(m, c.D, c.Q, le)
        cnt = _record_counts(R, L, nD, n)
        np.testing.assert_array_equal(np.bincount(ids, minlength=n), cnt)
        # query entries: the definition
        want_q = oracle.brute(m, c.D, c.Q, w, op, le_mask=le)
        qsel = ids >= nD
        np.testing.assert_array_equal(vals[qsel], want_q[ids[qsel] - nD])
        # data entries: the pair formula (the last axis compared with <: data
        # against data is the same for either tie rule)
        ww = np.ones(nD, dtype=np.int64) if op == "count" else c.w
        dt = _data_totals_by_pairs(m, c.D, ww, R, L, le, "max" if op == "max" else "sum", nD)
        for k in np.nonzero(~qsel)[0]:
            assert vals[k] == dt[ids[k]], (k, ids[k], vals[k], dt[ids[k]])


@pytest.mark.parametrize("m", [2, 3])
@pytest.mark.parametrize("op", ["max", "count", "sum"])
def test_final_list_shortcut_equals_general_for_monotone_f(m, op):
    c = _case(1300 + m, m, 200, 180, 9)
    w = None if op == "count" else np.abs(c.w)  # F(a, b) >= a: max, counts, sums of non-negatives
    a = oracle.final_list(m, c.D, c.Q, w, op)
    b = oracle.final_list(m, c.D, c.Q, w, op, shortcut=True)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_final_list_shortcut_differs_for_non_monotone_sum():
    """The shortcut's premise matters: with negative weights the running sum
    of an ID is not monotone and the maximum is not the total."""
    c = _case(1400, 2, 200, 180, 9)
    a = oracle.final_list(2, c.D, c.Q, c.w, "sum")
    b = oracle.final_list(2, c.D, c.Q, c.w, "sum", shortcut=True)
    assert not np.array_equal(a[1], b[1])


def test_final_list_basic_variant():
    c = _case(1500, 2, 60, 55, 5)
    ids, vals = oracle.final_list(2, c.D, c.Q, c.w, "sum", basic=True)
    _, E = oracle.construction_basic(2, c.D, c.Q, c.w, "sum", return_E=True)
    assert ids.size == E
    want = oracle.brute(2, c.D, c.Q, c.w, "sum")
    q = ids >= 60
    np.testing.assert_array_equal(vals[q], want[ids[q] - 60])


# --------------------------------------------------------------------------
# the multi-column Fenwick sweep (radix-sorted; the full-size pin for m = 2)


@pytest.mark.parametrize("alpha,coord", [(5, "int"), (None, "f32"), (40, "f32")])
def test_fenwick2_sums_equals_definition(alpha, coord):
    c = _case(1600 + (alpha or 0), 2, 700, 650, alpha, weight="f64", coord=coord)
    for le in range(4):
        s, sa, n1 = oracle.fenwick2_sums(c.D, c.Q, [c.w, np.abs(c.w), np.ones_like(c.w)], le_mask=le)
        np.testing.assert_allclose(s, oracle.brute(2, c.D, c.Q, c.w, "sum", le_mask=le), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(sa, oracle.brute(2, c.D, c.Q, np.abs(c.w), "sum", le_mask=le), rtol=1e-12)
        np.testing.assert_array_equal(n1, oracle.brute(2, c.D, c.Q, None, "count", le_mask=le))
        wi = (c.w * 100).astype(np.int64)
        np.testing.assert_array_equal(oracle.fenwick2_sums(c.D, c.Q, [wi], le_mask=le)[0],
                                      oracle.brute(2, c.D, c.Q, wi, "sum", le_mask=le))


def test_fenwick2_sums_negative_zero_infinities_and_empty():
    D = np.array([[-0.0, 1.0], [0.0, -np.inf], [np.inf, 0.0], [-1.0, -1.0]])
    Q = np.array([[0.0, 2.0], [np.inf, np.inf], [1e-30, 0.5], [-0.0, 3.0]])
    w = np.array([1.0, 2.0, 4.0, 8.0])
    np.testing.assert_array_equal(oracle.fenwick2_sums(D, Q, [w])[0], oracle.brute(2, D, Q, w, "sum"))
    assert oracle.fenwick2_sums(D[:0], Q, [w[:0]])[0].tolist() == [0.0] * 4
    assert oracle.fenwick2_sums(D, Q[:0], [w])[0].size == 0
