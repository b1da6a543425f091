"""The library without an allocator hook: plans, forward, backward,
recompute mode, graph replay, one-shot and batched calls, and plan
destruction, against the oracle.  Runs in a child process, since the Python
front end installs PyTorch's allocator as the hook on first use.

Skipped: a stream-ordered memory pool tried as the library's default
allocator (hipMallocFromPoolAsync / hipFreeAsync, hipFree at plan
destruction) left the GPU faulted in the run that first exercised it, with
every test and benchmark of that run passing; the cause was not found, the
pool was taken out (the default is hipMalloc / hipFree again), and this test
stays off until the default allocator is reworked and reviewed."""
import os
import subprocess
import sys

import pytest

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="the stream-ordered pool it was written for left the GPU faulted; "
                                      "taken out, cause not found (see the module docstring)")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys
import numpy as np
import torch
sys.path.insert(0, ROOT)
sys.path.insert(0, ROOT + "/tests")
import oracle, workloads
from gpu_helpers import check_exact, check_fp, to_dev
from paper_2305_16751_amd import DomAggPlan, dom_agg_run, binding

for rep in range(3):
    for m, n in ((2, 20000), (3, 3000)):
        c = workloads.small_case(3100 + m + rep, m, n, n - 55, alphabet=None, coord="f32", weight="int64")
        want = oracle.construction(m, c.D, c.Q, c.w, "sum")
        for flags in ({}, {"recompute": True}, {"graph": True}):
            p = DomAggPlan(to_dev(c.D), to_dev(c.Q), **flags)
            for _ in range(2):
                check_exact(p.forward(to_dev(c.w), "sum"), want, f"m={m} {flags}")
            g = np.random.default_rng(rep).standard_normal(c.Q.shape[0]).astype(np.float32)
            gw = oracle.transposed_sum(m, c.D, c.Q, g.astype(np.float64))
            gs = oracle.transposed_sum(m, c.D, c.Q, np.abs(g.astype(np.float64)))
            check_fp(p.backward(to_dev(g)), gw, gs, f"grad m={m} {flags}")
            p.close()
        w32 = (c.w % 1000).astype(np.int32)
        got = dom_agg_run(to_dev(c.D), to_dev(c.Q), to_dev(w32), "sum")
        check_exact(got, oracle.construction(m, c.D, c.Q, w32.astype(np.int64), "sum", weight_dtype=np.int32),
                    "one-shot")
rng = np.random.default_rng(3)
sizes = [500, 0, 900, 3]
Ds = [rng.integers(0, 70, size=(k, 2), dtype=np.int32) for k in sizes]
Qs = [rng.integers(0, 70, size=(k + 2, 2), dtype=np.int32) for k in sizes]
ws = [rng.integers(-9, 9, size=k).astype(np.int64) for k in sizes]
off = lambda xs: np.concatenate([[0], np.cumsum([x.shape[0] for x in xs])]).astype(np.int64)
got = dom_agg_run(to_dev(np.concatenate(Ds)), to_dev(np.concatenate(Qs)), to_dev(np.concatenate(ws)), "sum",
                  d_offsets=off(Ds), q_offsets=off(Qs))
check_exact(got, np.concatenate([oracle.construction(2, Ds[k], Qs[k], ws[k], "sum") for k in range(4)]), "batched")
torch.cuda.synchronize()
print("native pool ok")
'''


def test_library_pool_allocator():
    env = dict(os.environ)
    env["DOM_AGG_TORCH_ALLOC"] = "0"
    code = "ROOT = " + repr(ROOT) + "\n" + CHILD
    print("child process: library pool allocator", flush=True)
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "native pool ok" in r.stdout
