#!/usr/bin/env python3
"""Benchmark of dominance aggregation on one MI355X.

One step = the whole path on one batch of synthetic input: the coordinate
phase (ranks, flat map, record sort) plus the forward segmented scan and
regrouping, as one dom_agg_run call (the one-shot entry point, whose records
carry the weights), with inputs resident in HBM.  The reusable-plan path
(dom_agg_plan + dom_agg_forward) is timed too, as an extra.
Default workload: m = 2, |D| = |Q| = 2^24 float32 coordinates U[0,1), float32
weights N(0,1), F = sum (fp32 accumulation).

Prints one JSON line.  Per-kernel times come from HIP events the library
records around each launch on the stream it runs on; the roofline entry is
the record sort's onesweep pass (the dominant kernel).  The CPU baseline is
the oracle (plain sequential C of the paper's construction) timed on a
bounded sample of the same distribution.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "(|D|+|Q|)/s m=2,3 dominance sum; fwd+bwd & batched vs plain; HBM GB/s frac"
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def record_bytes(info, kernel=None):
    """Bytes of one sorted record: from the record-sort kernel's name when
    given (8 for records packed into one word, else key + 4-byte payload),
    else from the plan."""
    if kernel is not None:
        if "packed" in kernel:
            return 8
        return 12 if "_u64_" in kernel else 8
    return info["record_bytes"]


def record_sort_model(info, kernel=None):
    """Algorithmic bytes of the record sort and its number of digit passes:
    each pass reads and writes every record of its key-length class once."""
    rb = record_bytes(info, kernel)
    ncls = info["sort_classes"]
    total, launches = 0, 0
    for c, ec in enumerate(info["sort_class_records"]):
        passes = info["sort_passes"] - ncls + 1 + c
        if ec:
            total += passes * 2 * ec * rb
            launches += passes
    return total, launches


def stage_table(kern, steps, info, n, nax, wbytes=4):
    """Per-kernel average time and, where the kernel has a fixed algorithmic
    byte count, its achieved rate."""
    E = info["records"]
    ED = info["data_records"]
    EQ = E - ED
    rec = [k for k in kern if k.startswith("onesweep_records")]
    rb = record_bytes(info, rec[0] if rec else None)
    model = {
        "flatmap_emit": E * rb + n * (8 + 4 + 4 * nax),
        "forward_scan": E * rb + ED * wbytes + EQ * wbytes,
        # records that carry their weights: no weight gather
        "forward_scan_inline": E * rb + EQ * wbytes,
        "backward_scan": E * rb + EQ * wbytes + ED * wbytes,
    }
    out = {}
    for name, (ms, cnt) in sorted(kern.items(), key=lambda kv: -kv[1][0]):
        avg = ms / max(cnt, 1)
        row = {"ms_per_step": round(ms / steps, 4), "launches_per_step": round(cnt / steps, 2),
               "avg_ms_per_launch": round(avg, 5)}
        b = None
        if name.startswith("onesweep_records"):
            tot, launches = record_sort_model(info, name)
            b = tot / max(launches, 1)
        elif name in model:
            b = model[name]
        if b is not None and avg > 0:
            row["algorithmic_GB_per_launch"] = round(b / 1e9, 4)
            row["GBps"] = round(b / (avg * 1e-3) / 1e9, 1)
            row["frac_of_8TBps"] = round(b / (avg * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
        out[name] = row
    return out


def time_steps(fn, steps, warmup):
    import torch
    from paper_2305_16751_amd import binding
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    binding.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = binding.timing_read()
    binding.timing_enable(False)
    return (t1 - t0), kern


def run_oneshot(case, steps, warmup, op="sum"):
    """The headline step: one dom_agg_run call.  Plan info (sizes of the
    flat map and its classes) comes from a plan of the same points built
    outside the timed region."""
    import torch
    from paper_2305_16751_amd import DomAggPlan, dom_agg_run
    d = torch.from_numpy(case.D).cuda()
    q = torch.from_numpy(case.Q).cuda()
    w = torch.from_numpy(case.w).cuda()
    out = torch.empty(q.shape[0], dtype=torch.float32 if case.w.dtype == np.float32 else torch.int64,
                      device="cuda")
    p = DomAggPlan(d, q)
    info = p.info()
    p.close()

    def step():
        dom_agg_run(d, q, w, op, out=out)

    T, kern = time_steps(step, steps, warmup)
    return T, kern, info, out


def run_fwd_bwd(case, steps, warmup):
    """Plan + forward + backward (fp32 sums; the gradient of sum(c * out))
    per step, on one instance or a batch (case.d_offsets)."""
    import torch
    from paper_2305_16751_amd import DomAggPlan
    d = torch.from_numpy(case.D).cuda()
    q = torch.from_numpy(case.Q).cuda()
    w = torch.from_numpy(case.w).cuda()
    g = torch.from_numpy(case.c if getattr(case, "c", None) is not None else
                         np.random.default_rng(5).standard_normal(case.Q.shape[0]).astype(np.float32)).cuda()
    out = torch.empty(q.shape[0], device="cuda")
    gw = torch.empty(d.shape[0], device="cuda")
    offs = (case.d_offsets, case.q_offsets) if getattr(case, "d_offsets", None) is not None else (None, None)
    info = {}

    def step():
        p = DomAggPlan(d, q, *offs)
        p.forward(w, "sum", out=out)
        p.backward(g, out=gw)
        if not info:
            info.update(p.info())
        p.close()

    T, kern = time_steps(step, steps, warmup)
    return T, kern, info, out


def run_plain(case, steps, warmup, op="sum"):
    import torch
    from paper_2305_16751_amd import DomAggPlan
    d = torch.from_numpy(case.D).cuda()
    q = torch.from_numpy(case.Q).cuda()
    w = torch.from_numpy(case.w).cuda()
    out = torch.empty(q.shape[0], dtype=torch.float32 if case.w.dtype == np.float32 else torch.int64,
                      device="cuda")
    info = {}

    def step():
        plan = DomAggPlan(d, q)
        plan.forward(w, op, out=out)
        if not info:
            info.update(plan.info())
        plan.close()

    T, kern = time_steps(step, steps, warmup)
    return T, kern, info, out


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy), or None
    when there is none for this kernel or its sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic-record:"):
            rec = dict(kv.split("=", 1) for kv in line.split(":", 1)[1].split())
    if not rec or rec.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    for f in ("radix_sort.hpp", "device_common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2305_16751_amd", "csrc", f), "rb").read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return int(rec["bytes_per_launch"])


def roofline_entry(kern, info, workload=None):
    rec = {k: v for k, v in kern.items() if k.startswith("onesweep_records")}
    if not rec:
        return None
    name, (ms, cnt) = max(rec.items(), key=lambda kv: kv[1][0])
    avg_s = ms / cnt * 1e-3
    tot, launches = record_sort_model(info, name)
    b = tot / launches
    ach = b / avg_s / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": measured_traffic(name, workload) if workload else None,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "bytes_per_launch": round(b), "avg_launch_ms": round(avg_s * 1e3, 5),
            "bytes_model": "sum over key-length classes of passes_c * 2 * E_c * record bytes (8 when key and "
                           "payload are packed into one word, else key bytes + 4) (every record of a class "
                           "read and written once per pass of its class), divided by the number of passes"}


def _oracle_sample(args):
    """One core's share of the CPU baseline: the oracle's construction on its
    own seeded sample of the headline distribution (runs in a child process)."""
    n, seed = args
    import oracle
    import workloads
    c = workloads.f32_uniform(2, n, seed, "sample")
    w64 = c.w.astype(np.float64)
    t0 = time.perf_counter()
    oracle.construction(2, c.D, c.Q, w64, "sum")
    return 2 * n, time.perf_counter() - t0


def cpu_baseline(n_sample=1 << 20, cores=0):
    """The oracle on the host's cores: one independent sample per core, all
    at once (child processes, started fresh); the rate is the sum of the
    per-core rates."""
    import concurrent.futures
    import multiprocessing
    import workloads
    if cores <= 0:
        cores = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = multiprocessing.get_context("spawn")
    jobs = [(n_sample, workloads.BASE_SEED + 99 + i) for i in range(cores)]
    t0 = time.perf_counter()
    with concurrent.futures.ProcessPoolExecutor(max_workers=cores, mp_context=ctx) as ex:
        res = list(ex.map(_oracle_sample, jobs))
    wall = time.perf_counter() - t0
    rate = sum(p / dt for p, dt in res)
    dts = [dt for _, dt in res]
    return {"value": round(rate, 1), "unit": "(|D|+|Q|)/s", "cores": cores, "kind": "oracle",
            "sample": f"m=2, |D|=|Q|={n_sample} per core ({cores} independent samples run at once, one process "
                      f"each), float32 U[0,1) coordinates, float32 N(0,1) weights, fp64 sequential construction "
                      f"(Sec. 4 + Sec. 5); per-core time {min(dts):.2f}-{max(dts):.2f} s, {wall:.1f} s wall"}


def extra_plan_forward(case, steps, reps=10):
    """The reusable-plan path on the headline workload: dom_agg_plan +
    dom_agg_forward (payloads are indices, the scan gathers the weights);
    then dom_agg_forward alone on a kept plan, each call timed on its own
    (median and minimum of reps calls after 3 warm-up calls)."""
    import torch
    from paper_2305_16751_amd import DomAggPlan
    T, kern, info, _ = run_plain(case, steps, 2)
    d = torch.from_numpy(case.D).cuda()
    q = torch.from_numpy(case.Q).cuda()
    w = torch.from_numpy(case.w).cuda()
    out = torch.empty(q.shape[0], dtype=torch.float32, device="cuda")
    p = DomAggPlan(d, q)
    for _ in range(3):
        p.forward(w, "sum", out=out)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        p.forward(w, "sum", out=out)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    p.close()
    return {"workload": case.name, "value": round(case.n * steps / T, 1), "ms_per_step": round(T / steps * 1e3, 3),
            "step": "dom_agg_plan + dom_agg_forward",
            "forward_kept_plan_ms": {"median": round(float(np.median(times)), 3), "min": round(min(times), 3),
                                     "calls": reps},
            "stages": stage_table(kern, steps, info, case.n, case.m - 1)}


def extra_m3(steps):
    import workloads
    c = workloads.f32_3d_1m()
    T, kern, info, _ = run_oneshot(c, steps, 2)
    return {"workload": "f32_3d_1m", "value": round(c.n * steps / T, 1), "ms_per_step": round(T / steps * 1e3, 3),
            "records": info["records"], "key_bits": info["key_bits"],
            "stages": stage_table(kern, steps, info, c.n, 2)}


def extra_fwd_bwd(steps):
    import torch
    import workloads
    from paper_2305_16751_amd import DomAggPlan
    c = workloads.f32_2d_4m_grad()
    d = torch.from_numpy(c.D).cuda()
    q = torch.from_numpy(c.Q).cuda()
    w = torch.from_numpy(c.w).cuda()
    g = torch.from_numpy(c.c).cuda()
    out = torch.empty(q.shape[0], device="cuda")
    gw = torch.empty(d.shape[0], device="cuda")

    def fwd():
        p = DomAggPlan(d, q)
        p.forward(w, "sum", out=out)
        p.close()

    def fwd_bwd():
        p = DomAggPlan(d, q)
        p.forward(w, "sum", out=out)
        p.backward(g, out=gw)
        p.close()

    Tf, _ = time_steps(fwd, steps, 2)
    Tb, kern = time_steps(fwd_bwd, steps, 2)
    return {"workload": "f32_2d_4m_grad", "fwd_ms": round(Tf / steps * 1e3, 3),
            "fwd_bwd_ms": round(Tb / steps * 1e3, 3), "ratio": round(Tb / Tf, 3),
            "backward_scan_ms": round(kern.get("backward_scan", (0, 1))[0] / steps, 4)}


def _replay_ms(fn, reps):
    """Average ms of fn() over reps calls (after one warm call), bracketed by
    synchronisations."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3


def extra_batched(reps):
    """4096 independent m = 2 instances (int coordinates, int64 weights, sum):
    one batched plan + graph-replayed forward per step, against launching
    plan + forward once per instance; plus the forward alone, replayed from
    the kept plan's graph."""
    import torch
    import workloads
    from paper_2305_16751_amd import DomAggPlan
    c = workloads.batched_int2d()
    d = torch.from_numpy(c.D).cuda()
    q = torch.from_numpy(c.Q).cuda()
    w = torch.from_numpy(c.w).cuda()
    out = torch.empty(q.shape[0], dtype=torch.int64, device="cuda")

    def batched():
        p = DomAggPlan(d, q, c.d_offsets, c.q_offsets, graph=True)
        p.forward(w, "sum", out=out)
        p.close()

    Tb, kern = time_steps(batched, reps, 1)
    kept = DomAggPlan(d, q, c.d_offsets, c.q_offsets, graph=True)
    info = kept.info()
    fwd_ms = _replay_ms(lambda: kept.forward(w, "sum", out=out), 10)
    kept.close()
    doff, qoff = c.d_offsets, c.q_offsets

    def per_instance():
        for k in range(len(doff) - 1):
            p = DomAggPlan(d[doff[k]:doff[k + 1]], q[qoff[k]:qoff[k + 1]])
            p.forward(w[doff[k]:doff[k + 1]], "sum", out=out[qoff[k]:qoff[k + 1]])
            p.close()

    Tp, _ = time_steps(per_instance, 1, 1)
    tb, tp = Tb / reps, Tp
    return {"workload": "batched_int2d", "instances": len(doff) - 1, "points": c.n, "records": info["records"],
            "batched_ms": round(tb * 1e3, 3), "per_instance_ms": round(tp * 1e3, 3),
            "batched_value": round(c.n / tb, 1), "per_instance_value": round(c.n / tp, 1),
            "speedup": round(tp / tb, 2), "forward_replay_ms": round(fwd_ms, 3),
            "stages": stage_table(kern, reps, info, c.n, 1, wbytes=8)}


def extra_batched_gmm4d(reps):
    """64 independent m = 4 instances (Gaussian-mixture points, fp32 weights):
    batched plan + forward, plan + forward + backward (the fwd+bwd ratio),
    the forward and backward alone replayed from the kept plan's graphs,
    int32 max, and plan + forward launched once per instance."""
    import torch
    import workloads
    from paper_2305_16751_amd import DomAggPlan
    c = workloads.batched_gmm4d()
    d = torch.from_numpy(c.D).cuda()
    q = torch.from_numpy(c.Q).cuda()
    w = torch.from_numpy(c.w).cuda()
    wi = torch.from_numpy(c.w_alt).cuda()
    g = torch.from_numpy(np.random.default_rng(5).standard_normal(c.Q.shape[0]).astype(np.float32)).cuda()
    out = torch.empty(q.shape[0], device="cuda")
    outi = torch.empty(q.shape[0], dtype=torch.int32, device="cuda")
    gw = torch.empty(d.shape[0], device="cuda")
    doff, qoff = c.d_offsets, c.q_offsets

    def fwd():
        p = DomAggPlan(d, q, doff, qoff, graph=True)
        p.forward(w, "sum", out=out)
        p.close()

    def fwd_bwd():
        p = DomAggPlan(d, q, doff, qoff, graph=True)
        p.forward(w, "sum", out=out)
        p.backward(g, out=gw)
        p.close()

    Tf, kern = time_steps(fwd, reps, 1)
    Tb, _ = time_steps(fwd_bwd, reps, 1)
    kept = DomAggPlan(d, q, doff, qoff, graph=True)
    info = kept.info()
    fwd_ms = _replay_ms(lambda: kept.forward(w, "sum", out=out), 5)
    bwd_ms = _replay_ms(lambda: kept.backward(g, out=gw), 5)
    max_ms = _replay_ms(lambda: kept.forward(wi, "max", out=outi), 5)
    kept.close()

    def per_instance():
        for k in range(len(doff) - 1):
            p = DomAggPlan(d[doff[k]:doff[k + 1]], q[qoff[k]:qoff[k + 1]])
            p.forward(w[doff[k]:doff[k + 1]], "sum", out=out[qoff[k]:qoff[k + 1]])
            p.close()

    Tp, _ = time_steps(per_instance, 1, 1)
    tf, tb, tp = Tf / reps, Tb / reps, Tp
    return {"workload": "batched_gmm4d", "instances": len(doff) - 1, "points": c.n, "records": info["records"],
            "key_bits": info["key_bits"], "regroup": "slots" if info["regroup_slots"] else "compact",
            "plan_fwd_ms": round(tf * 1e3, 3), "value": round(c.n / tf, 1),
            "plan_fwd_bwd_ms": round(tb * 1e3, 3), "fwd_bwd_ratio": round(tb / tf, 3),
            "forward_replay_ms": round(fwd_ms, 3), "backward_replay_ms": round(bwd_ms, 3),
            "max_int32_replay_ms": round(max_ms, 3),
            "per_instance_ms": round(tp * 1e3, 3), "per_instance_value": round(c.n / tp, 1),
            "speedup": round(tp / tf, 2),
            "stages": stage_table(kern, reps, info, c.n, 3)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="only the headline workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20, help="points per side of each core's sample")
    ap.add_argument("--cpu-cores", type=int, default=0, help="cores for the CPU baseline (0: up to 16 available)")
    ap.add_argument("--workload", choices=("f32_2d_16m", "f32_3d_1m", "f32_2d_4m_grad", "batched_gmm4d"),
                    default="f32_2d_16m",
                    help="the workload of the JSON line (for profiling the others; the metric's workload is "
                         "f32_2d_16m): one-shot calls for the first two, plan + forward + backward for the "
                         "last two")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB elementwise copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    # the CPU baseline first: its worker processes start before this process
    # touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on the host cores) ...")
        cpu = cpu_baseline(args.cpu_sample, args.cpu_cores)
        log(f"cpu baseline: {json.dumps(cpu)}")

    import torch
    import workloads
    assert torch.cuda.is_available(), "no GPU"
    log(f"device: {torch.cuda.get_device_name(0)}")

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.add(a, 0.0, out=b)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b
    case = getattr(workloads, args.workload)()
    log(f"headline: {case.name} m={case.m} |D|={case.D.shape[0]} |Q|={case.Q.shape[0]}")
    fwd_bwd = args.workload in ("f32_2d_4m_grad", "batched_gmm4d")
    if fwd_bwd:
        T, kern, info, _ = run_fwd_bwd(case, args.steps, args.warmup)
    else:
        T, kern, info, _ = run_oneshot(case, args.steps, args.warmup)
    value = case.n * args.steps / T
    log(f"headline: {T / args.steps * 1e3:.3f} ms/step, {value:.4g} (|D|+|Q|)/s, E={info['records']}")
    result = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "(|D|+|Q|)/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(T / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "m": case.m, "n_data": int(case.D.shape[0]),
                   "n_query": int(case.Q.shape[0]), "op": "sum",
                   "coords": ("per-instance Gaussian mixtures" if case.name == "batched_gmm4d"
                              else "float32 U[0,1)"),
                   "weights": "float32 N(0,1)", "records": info["records"], "key_bits": info["key_bits"],
                   "sort_passes": info["sort_passes"], "sort_classes": info["sort_classes"], "sort_tile": info["sort_tile"],
                   "scan_tile": info["scan_tile"],
                   "step": ("dom_agg_plan + dom_agg_forward + dom_agg_backward" if fwd_bwd
                            else "dom_agg_run (plan + forward in one call)")},
        "roofline": roofline_entry(kern, info, case.name),
    }
    extra = {"stages": stage_table(kern, args.steps, info, case.n, case.m - 1)}
    if cpu is not None:
        result["cpu_baseline"] = cpu
    if not args.no_extras:
        for name, fn in (("plan_forward", lambda: extra_plan_forward(case, 5)), ("m3", lambda: extra_m3(5)),
                         ("fwd_bwd", lambda: extra_fwd_bwd(5)), ("batched", lambda: extra_batched(3)),
                         ("batched_gmm4d", lambda: extra_batched_gmm4d(3))):
            log(f"extra: {name} ...")
            try:
                extra[name] = fn()
            except Exception as e:  # an extra must not hide the headline line
                extra[name] = {"error": repr(e)}
            log(f"extra: {name}: {json.dumps(extra[name])[:300]}")
    result["extra"] = extra
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
