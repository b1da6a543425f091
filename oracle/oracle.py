"""ctypes wrapper around the oracle's C code (test infrastructure only).

Each function takes numpy arrays on the host and returns numpy arrays.
Coordinates are converted to float64 (exact for int32 and float32 inputs).
Float weights are accumulated in float64, integer weights in int64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ["dom_agg_oracle.c", "fenwick_pin.c", "cdq3_pin.c"]
_LIB_NAME = "liboracle.so"

SUM, MAX, COUNT = 0, 1, 2
_OPS = {"sum": SUM, "max": MAX, "count": COUNT}


class OracleError(RuntimeError):
    pass


def lib_path() -> str:
    return os.path.join(_HERE, _LIB_NAME)


def build() -> str:
    """Compile the oracle's C sources with gcc into oracle/liboracle.so."""
    out = lib_path()
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp] + [os.path.join(_HERE, s) for s in _SOURCES] + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    I = ctypes.c_int
    D = ctypes.c_double
    lib.oracle_brute_f64.argtypes = [I, I64, P, I64, P, P, I, D, P]
    lib.oracle_brute_i64.argtypes = [I, I64, P, I64, P, P, I, I64, P]
    lib.oracle_dom_agg_f64.argtypes = [I, I64, P, I64, P, P, I, D, P, P, P]
    lib.oracle_dom_agg_i64.argtypes = [I, I64, P, I64, P, P, I, I64, P, P, P]
    lib.oracle_dom_agg_basic_f64.argtypes = [I, I64, P, I64, P, P, I, D, P, P]
    lib.oracle_dom_agg_basic_i64.argtypes = [I, I64, P, I64, P, P, I, I64, P, P]
    lib.oracle_transposed_sum_f64.argtypes = [I, I64, P, I64, P, P, P]
    lib.oracle_sscan_f64.argtypes = [I64, P, P, I, P]
    lib.oracle_prefix_set.argtypes = [ctypes.c_uint64, I, I, P, P]
    lib.oracle_dense_rank.argtypes = [I64, P, P, P]
    lib.oracle_bits_for.argtypes = [I64]
    lib.pin_fenwick2_f64.argtypes = [I64, P, I64, P, P, I, D, P]
    lib.pin_fenwick2_i64.argtypes = [I64, P, I64, P, P, I, I64, P]
    lib.pin_cdq3_f64.argtypes = [I64, P, I64, P, P, I, D, I, P]
    lib.pin_fenwick2_multi.argtypes = [I64, P, I64, P, I, P, I, I, P]
    lib.pin_cdq3_i64.argtypes = [I64, P, I64, P, P, I, I64, I, P]
    lib.oracle_brute_le_f64.argtypes = [I, I64, P, I64, P, P, I, D, I, P]
    lib.oracle_brute_le_i64.argtypes = [I, I64, P, I64, P, P, I, I64, I, P]
    lib.oracle_dom_agg_ex_f64.argtypes = [I, I64, P, I64, P, P, I, D, I, I, P, P, P, P, P, I64, I]
    lib.oracle_dom_agg_ex_i64.argtypes = [I, I64, P, I64, P, P, I, I64, I, I, P, P, P, P, P, I64, I]
    lib.oracle_transposed_sum_le_f64.argtypes = [I, I64, P, I64, P, P, I, P]
    for name in ("oracle_brute_f64", "oracle_brute_i64", "oracle_dom_agg_f64",
                 "oracle_dom_agg_i64", "oracle_dom_agg_basic_f64",
                 "oracle_dom_agg_basic_i64", "oracle_transposed_sum_f64",
                 "oracle_sscan_f64", "oracle_prefix_set", "oracle_dense_rank",
                 "oracle_bits_for", "pin_fenwick2_f64", "pin_fenwick2_i64",
                 "pin_cdq3_f64", "pin_cdq3_i64", "pin_fenwick2_multi", "oracle_brute_le_f64", "oracle_brute_le_i64",
                 "oracle_dom_agg_ex_f64", "oracle_dom_agg_ex_i64", "oracle_transposed_sum_le_f64"):
        getattr(lib, name).restype = I
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def _coords(x, m):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64)).reshape(-1, m)
    return x


def _check(rc, what):
    if rc == -2:
        raise OracleError(f"{what}: NaN coordinate")
    if rc == -4:
        raise OracleError(f"{what}: output list too short")
    if rc != 0:
        raise OracleError(f"{what}: error {rc}")


def identity(op: str, weight_dtype) -> float | int:
    """The unit e of F for a weight dtype: 0 for sum and count, the dtype's
    minimum (-inf for floats) for max."""
    dt = np.dtype(weight_dtype)
    if op in ("sum", "count"):
        return 0
    if dt.kind == "f":
        return -np.inf
    return int(np.iinfo(dt).min)


def _weights(w, op, nD, weight_dtype):
    """Returns (weights as float64 or int64, is_float, the dtype whose unit e
    applies)."""
    if op == "count":
        return None, False, np.dtype(np.int64)
    if w is None:
        raise OracleError("weights required for sum and max")
    w = np.asarray(w)
    src = np.dtype(weight_dtype) if weight_dtype is not None else w.dtype
    is_float = w.dtype.kind == "f"
    w = np.ascontiguousarray(w, dtype=np.float64 if is_float else np.int64)
    if w.shape != (nD,):
        raise OracleError("weights must have shape [nD]")
    return w, is_float, src


def _run(kind, m, D, Q, w, op, weight_dtype=None, le_mask=0, agg=False, shortcut=False):
    """kind: 'brute' (the definition), 'sec5' (the construction with the
    Sec. 5 improvement) or 'basic' (the basic construction of Sec. 4)."""
    lib = _load()
    D = _coords(D, m)
    Q = _coords(Q, m)
    nD, nQ = D.shape[0], Q.shape[0]
    w, is_float, wd = _weights(w, op, nD, weight_dtype)
    e = identity(op, wd)
    E = ctypes.c_int64(0)
    L = (ctypes.c_int * 8)()
    vt = np.float64 if is_float else np.int64
    out = np.empty(nQ, dtype=vt)
    ids = vals = None
    if kind == "brute":
        fn = lib.oracle_brute_le_f64 if is_float else lib.oracle_brute_le_i64
        ev = float(e) if is_float else int(e)
        rc = fn(m, nD, _ptr(D), nQ, _ptr(Q), _ptr(w), _OPS[op], ev, int(le_mask), _ptr(out))
    else:
        fn = lib.oracle_dom_agg_ex_f64 if is_float else lib.oracle_dom_agg_ex_i64
        ev = float(e) if is_float else int(e)
        sec5 = 1 if kind == "sec5" else 0
        cap = 0
        if agg:
            # the size of the final list is E: one run of the construction to learn it
            rc = fn(m, nD, _ptr(D), nQ, _ptr(Q), _ptr(w), _OPS[op], ev, sec5, int(le_mask), _ptr(out),
                    ctypes.byref(E), L, None, None, 0, 0)
            _check(rc, kind)
            cap = int(E.value)
            ids = np.empty(cap, dtype=np.int64)
            vals = np.empty(cap, dtype=vt)
        rc = fn(m, nD, _ptr(D), nQ, _ptr(Q), _ptr(w), _OPS[op], ev, sec5, int(le_mask), _ptr(out),
                ctypes.byref(E), L, _ptr(ids) if agg else None, _ptr(vals) if agg else None, cap,
                1 if shortcut else 0)
    _check(rc, kind)
    nL = max(m - 1, 0) if kind == "sec5" else m
    return out, int(E.value), [int(L[i]) for i in range(nL)], ids, vals


def brute(m, D, Q, w=None, op="sum", weight_dtype=None, le_mask=0):
    """Plain definition (Sec. 1.2): for each query, F over the weights of the
    data points it strictly dominates (or dominates with <= on the axes whose
    bit is set in le_mask).  O(|D||Q|m)."""
    return _run("brute", m, D, Q, w, op, weight_dtype, le_mask)[0]


def construction(m, D, Q, w=None, op="sum", weight_dtype=None, return_stats=False, le_mask=0):
    """The paper's construction with the Sec. 5 improvement.  With
    return_stats, also returns (E, L): the expanded record count and the bit
    width of each expanded axis."""
    out, E, L, _, _ = _run("sec5", m, D, Q, w, op, weight_dtype, le_mask)
    return (out, E, L) if return_stats else out


def construction_basic(m, D, Q, w=None, op="sum", weight_dtype=None, return_E=False, le_mask=0,
                       return_stats=False):
    """The basic construction of Sec. 4 (all m axes expanded)."""
    out, E, L, _, _ = _run("basic", m, D, Q, w, op, weight_dtype, le_mask)
    if return_stats:
        return out, E, L
    return (out, E) if return_E else out


def final_list(m, D, Q, w=None, op="sum", weight_dtype=None, le_mask=0, shortcut=False, basic=False):
    """The list the last instructions of Sec. 4 build: (ids, vals), E entries
    in nondecreasing ID order (data IDs 0..|D|-1, then queries |D|..), each
    ID once per record of its point, each value the total of its ID.
    shortcut: built by the segmented broadcast of the maximum instead (valid
    when F(a, b) >= a)."""
    _, _, _, ids, vals = _run("basic" if basic else "sec5", m, D, Q, w, op, weight_dtype, le_mask,
                              agg=True, shortcut=shortcut)
    return ids, vals


def transposed_sum(m, D, Q, g, le_mask=0):
    """grad[i] = sum of g[j] over queries j that dominate D[i] (strictly, or
    with <= on the axes of le_mask)."""
    lib = _load()
    D = _coords(D, m)
    Q = _coords(Q, m)
    g = np.ascontiguousarray(g, dtype=np.float64)
    grad = np.empty(D.shape[0], dtype=np.float64)
    rc = lib.oracle_transposed_sum_le_f64(m, D.shape[0], _ptr(D), Q.shape[0], _ptr(Q), _ptr(g), int(le_mask),
                                          _ptr(grad))
    _check(rc, "transposed_sum")
    return grad


def sscan(a, t, op="sum"):
    """Segmented inclusive scan of a, segments = maximal runs of equal t."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.int64)
    out = np.empty_like(a)
    _check(lib.oracle_sscan_f64(a.size, _ptr(a), _ptr(t), _OPS[op], _ptr(out)), "sscan")
    return out


def prefix_set(x: int, L: int, bit: int):
    """P0 (bit=0) or P1 (bit=1) of the L-bit string of x, as bitstrings."""
    lib = _load()
    lens = np.zeros(64, dtype=np.int32)
    vals = np.zeros(64, dtype=np.uint64)
    c = lib.oracle_prefix_set(x, L, bit, _ptr(lens), _ptr(vals))
    if c < 0:
        raise OracleError("prefix_set: bad argument")
    return [format(int(vals[i]), "0%db" % lens[i]) if lens[i] else "" for i in range(c)]


def dense_rank(v):
    lib = _load()
    v = np.ascontiguousarray(v, dtype=np.float64)
    r = np.empty(v.size, dtype=np.int64)
    K = ctypes.c_int64(0)
    _check(lib.oracle_dense_rank(v.size, _ptr(v), _ptr(r), ctypes.byref(K)), "dense_rank")
    return r, int(K.value)


def bits_for(K: int) -> int:
    return int(_load().oracle_bits_for(K))


def fenwick2(D, Q, w=None, op="sum", weight_dtype=None):
    """Textbook sweep + Fenwick tree for m = 2 (a pin, not the construction)."""
    lib = _load()
    D = _coords(D, 2)
    Q = _coords(Q, 2)
    nD, nQ = D.shape[0], Q.shape[0]
    if op == "count":
        w = np.ones(nD, dtype=np.int64)
        op_ = "sum"
    else:
        op_ = op
    w, is_float, wd = _weights(w, op_, nD, weight_dtype)
    e = identity(op_, wd)
    if is_float:
        out = np.empty(nQ, dtype=np.float64)
        rc = lib.pin_fenwick2_f64(nD, _ptr(D), nQ, _ptr(Q), _ptr(w), int(op_ == "max"), float(e), _ptr(out))
    else:
        out = np.empty(nQ, dtype=np.int64)
        rc = lib.pin_fenwick2_i64(nD, _ptr(D), nQ, _ptr(Q), _ptr(w), int(op_ == "max"), int(e), _ptr(out))
    _check(rc, "fenwick2")
    return out


def sweep(m, D, Q, w=None, op="sum", weight_dtype=None, le_mask=0):
    """Textbook offline divide and conquer for m <= 3 (a pin, not the
    construction): sort by the first axis, split in halves, settle the pairs
    across the halves while merging by the second axis with a Fenwick tree
    over ranks of the third.  Smaller m pad constant axes compared with <=."""
    if m > 3:
        raise OracleError("sweep: m <= 3")
    lib = _load()
    D = _coords(D, m)
    Q = _coords(Q, m)
    nD, nQ = D.shape[0], Q.shape[0]
    if m < 3:
        D = np.ascontiguousarray(np.hstack([D, np.zeros((nD, 3 - m))]))
        Q = np.ascontiguousarray(np.hstack([Q, np.zeros((nQ, 3 - m))]))
        le_mask = int(le_mask) | sum(1 << a for a in range(m, 3))
    if op == "count":
        w = np.ones(nD, dtype=np.int64)
        op_ = "sum"
    else:
        op_ = op
    w, is_float, wd = _weights(w, op_, nD, weight_dtype)
    e = identity(op_, wd)
    if is_float:
        out = np.empty(nQ, dtype=np.float64)
        rc = lib.pin_cdq3_f64(nD, _ptr(D), nQ, _ptr(Q), _ptr(w), int(op_ == "max"), float(e), int(le_mask), _ptr(out))
    else:
        out = np.empty(nQ, dtype=np.int64)
        rc = lib.pin_cdq3_i64(nD, _ptr(D), nQ, _ptr(Q), _ptr(w), int(op_ == "max"), int(e), int(le_mask), _ptr(out))
    _check(rc, "sweep")
    return out


def fenwick2_sums(D, Q, columns, le_mask=0):
    """The m = 2 textbook sweep for several weight columns in one pass (sums
    only; a pin at tens of millions of points).  columns: list of [|D|]
    arrays, all float or all integer; returns one [|Q|] array per column
    (float64 or int64)."""
    lib = _load()
    D = _coords(D, 2)
    Q = _coords(Q, 2)
    nD, nQ = D.shape[0], Q.shape[0]
    is_int = all(np.asarray(c).dtype.kind in "iub" for c in columns)
    vt = np.int64 if is_int else np.float64
    W = np.ascontiguousarray(np.stack([np.asarray(c, dtype=vt) for c in columns]) if nD else
                             np.zeros((len(columns), 0), dtype=vt))
    if W.shape != (len(columns), nD):
        raise OracleError("columns must have shape [nD]")
    out = np.empty((len(columns), nQ), dtype=vt)
    rc = lib.pin_fenwick2_multi(nD, _ptr(D), nQ, _ptr(Q), len(columns), _ptr(W), int(is_int), int(le_mask),
                                _ptr(out))
    _check(rc, "fenwick2_sums")
    return [out[i] for i in range(len(columns))]
