"""Aggregation over dominated points on AMD Instinct MI355X (gfx950).

The paper's construction (Sroka & Tyszkiewicz, arXiv 2305.16751, Sec. 4 with
the Sec. 5 improvement) as hand-written HIP kernels behind the C-ABI of
include/dom_agg.h; this package is its PyTorch front end.
"""
from .binding import DomAggError  # noqa: F401
from .dom_agg import DomAggFunction, DomAggPlan, dom_agg, dom_agg_batched, dom_agg_run  # noqa: F401
