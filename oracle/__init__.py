"""CPU oracle for aggregation over dominated points.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.

It wraps the plain C of ``dom_agg_oracle.c`` (the paper's construction of
Sec. 4 with the Sec. 5 improvement, its basic Sec. 4 variant and the plain
definition of Sec. 1.2) and the textbook sweeps ``fenwick_pin.c`` (m = 2) and
``cdq3_pin.c`` (m <= 3, divide and conquer), used only as pins.  Arithmetic is fp64 for float weights and
int64 for integer weights.
"""
from .oracle import (  # noqa: F401
    OracleError,
    brute,
    construction,
    construction_basic,
    transposed_sum,
    sscan,
    prefix_set,
    dense_rank,
    bits_for,
    fenwick2,
    fenwick2_sums,
    sweep,
    final_list,
    identity,
    build,
    lib_path,
)
