"""The size limits of a plan on the GPU: a record key wider than 64 bits and
a flat map of more than 2^32 - 2^20 records are rejected with ETOOBIG before
any record is written (the first after the ranks, the second after the
count pass), by the plan and by the one-shot call alike."""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV

pytestmark = pytest.mark.gpu


def _expect_toobig(D, Q, what):
    from paper_2305_16751_amd import DomAggError, DomAggPlan, dom_agg_run
    d = torch.from_numpy(D).to(DEV)
    q = torch.from_numpy(Q).to(DEV)
    with pytest.raises(DomAggError, match="ETOOBIG") as e:
        DomAggPlan(d, q)
    assert what in str(e.value), str(e.value)
    with pytest.raises(DomAggError, match="ETOOBIG"):
        dom_agg_run(d, q, torch.ones(D.shape[0], device=DEV), "sum")
    # the library is still usable afterwards
    small = DomAggPlan(d[:100], q[:100])
    assert small.forward(None, "count").shape[0] == 100


def test_key_wider_than_64_bits():
    """m = 4 with 2^21 + 2^21 distinct values per axis: 22 digits on each of
    the three expanded axes, 66 key bits."""
    rng = np.random.default_rng(11)
    n = 1 << 21
    cols = [rng.permutation(np.arange(2 * n, dtype=np.int32)) for _ in range(4)]
    P = np.stack(cols, 1)
    print("limits: 66-bit keys", flush=True)
    _expect_toobig(P[:n].copy(), P[n:].copy(), "bits")


def test_more_records_than_the_limit():
    """m = 4, K = 2^21 distinct values per axis (21 digits): data points at
    the smallest value (rank 0, every digit 0) and queries at the largest
    (rank 2^21 - 1, every digit 1) each yield 21^3 records, so 320k of each
    need 5.9e9 records, more than 2^32 - 2^20."""
    rng = np.random.default_rng(12)
    K = 1 << 21
    filler = np.stack([rng.permutation(np.arange(K, dtype=np.int32)) for _ in range(4)], 1)
    k = 320_000
    lowD = np.zeros((k, 4), dtype=np.int32)
    highQ = np.full((k, 4), K - 1, dtype=np.int32)
    D = np.concatenate([filler[: K // 2], lowD])
    Q = np.concatenate([filler[K // 2:], highQ])
    print("limits: 5.9e9 records", flush=True)
    _expect_toobig(D, Q, "records")
