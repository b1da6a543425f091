"""bench.py's host-side logic without a GPU: the one-GPU contract, the byte
model behind the roofline figure, the traffic record of the committed
counter summary, and the CPU baseline on a tiny sample."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_record_bytes_from_kernel_names():
    assert bench.record_bytes({}, "onesweep_records_packed_t8192") == 8
    assert bench.record_bytes({}, "onesweep_records_packed_t8192_d7") == 8
    assert bench.record_bytes({}, "onesweep_records_u32_t4096") == 8
    assert bench.record_bytes({}, "onesweep_records_u64_t4096") == 12
    assert bench.record_bytes({"record_bytes": 12}) == 12


def test_record_sort_model_sums_classes():
    """Class c of C is sorted with sort_passes - C + 1 + c passes; every pass
    reads and writes each of its records once."""
    info = {"sort_classes": 3, "sort_passes": 3, "sort_class_records": [100, 200, 300, 0]}
    total, launches = bench.record_sort_model(info, "onesweep_records_packed_t8192")
    assert launches == 1 + 2 + 3
    assert total == (1 * 100 + 2 * 200 + 3 * 300) * 2 * 8
    # one class: all records, sort_passes passes
    info1 = {"sort_classes": 1, "sort_passes": 4, "sort_class_records": [1000, 0, 0, 0]}
    assert bench.record_sort_model(info1, "onesweep_records_u64_t4096") == (4 * 1000 * 2 * 12, 4)
    # empty classes launch nothing
    info2 = {"sort_classes": 2, "sort_passes": 2, "sort_class_records": [0, 50, 0, 0]}
    assert bench.record_sort_model(info2, "onesweep_records_packed_t8192") == (2 * 50 * 2 * 8, 2)


def test_traffic_record_follows_the_sources():
    """The committed counter summary's traffic record is reported only while
    the sort's sources hash to the value recorded with it."""
    path = os.path.join(ROOT, "profiles", "f32_2d_16m_hbm_traffic.md")
    rec = None
    for line in open(path):
        if line.startswith("traffic-record:"):
            rec = dict(kv.split("=", 1) for kv in line.split(":", 1)[1].split())
    assert rec is not None
    h = hashlib.sha256()
    for f in ("radix_sort.hpp", "device_common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2305_16751_amd", "csrc", f), "rb").read())
    got = bench.measured_traffic(rec["kernel"], "f32_2d_16m")
    if h.hexdigest() == rec["sources_sha256"]:
        assert got == int(rec["bytes_per_launch"])
        assert abs(got - int(rec["fetch"]) - int(rec["write"])) <= 1  # (each truncated to whole bytes)
    else:
        assert got is None
    assert bench.measured_traffic("no_such_kernel", "f32_2d_16m") is None
    assert bench.measured_traffic(rec["kernel"], "no_such_workload") is None


def test_cpu_baseline_shape():
    cb = bench.cpu_baseline(1 << 10, 2)
    assert cb["kind"] == "oracle" and cb["cores"] == 2 and cb["unit"] == "(|D|+|Q|)/s"
    assert cb["value"] > 0
    assert "per core" in cb["sample"]


def test_stage_table_forward_scan_models():
    """The forward scan gathers one weight per data record, unless the
    records carry the weights (the one-shot call's own launch name); both
    store one partial per query record."""
    E, ED = 400_000_000, 160_000_000
    info = {"records": E, "data_records": ED, "record_bytes": 8, "sort_classes": 1, "sort_passes": 2,
            "sort_class_records": [E, 0, 0, 0]}
    kern = {"forward_scan": (2.0, 1), "forward_scan_inline": (1.0, 1), "onesweep_records_packed_t8192": (4.0, 2)}
    st = bench.stage_table(kern, 1, info, 100, 1)
    gb = lambda k: st[k]["algorithmic_GB_per_launch"] * 1e9
    assert gb("forward_scan") == pytest.approx(E * 8 + ED * 4 + (E - ED) * 4, rel=1e-4)
    assert gb("forward_scan_inline") == pytest.approx(E * 8 + (E - ED) * 4, rel=1e-4)
    # the sort: two passes over E packed records, each read and written once per pass
    assert gb("onesweep_records_packed_t8192") == pytest.approx(2 * E * 8, rel=1e-4)
    assert st["forward_scan_inline"]["GBps"] == pytest.approx((E * 8 + (E - ED) * 4) / 1e-3 / 1e9, rel=1e-4)


def test_stage_model_names_are_launch_names():
    """Every stage the byte model prices is a name the library times its
    launches under (a renamed launch would silently drop its rate), and so
    is every record-sort name the roofline figure can be quoted on."""
    src = open(os.path.join(ROOT, "paper_2305_16751_amd", "csrc", "dom_agg.hip")).read()
    info = {"records": 10, "data_records": 4, "record_bytes": 8, "sort_classes": 1, "sort_passes": 1,
            "sort_class_records": [10, 0, 0, 0]}
    for name in ("flatmap_emit", "forward_scan", "forward_scan_inline", "backward_scan"):
        assert bench.stage_table({name: (1.0, 1)}, 1, info, 1, 1)[name].get("algorithmic_GB_per_launch") is not None
        assert f'"{name}"' in src, name
    for name in ("onesweep_records_packed_t8192", "onesweep_records_packed_t8192_d7", "onesweep_records_u64_t4096",
                 "onesweep_records_u32_t8192"):
        assert f'"{name}"' in src, name
