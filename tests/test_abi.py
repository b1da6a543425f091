"""The C-ABI library loads, exports every symbol include/dom_agg.h declares,
and rejects invalid arguments before touching the GPU.  No GPU needed: every
call here either fails validation or (with valid arguments and no device)
reports ENODEV."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dom_agg.h")


@pytest.fixture(scope="module")
def B():
    from paper_2305_16751_amd import binding
    from paper_2305_16751_amd.build import lib_path, build
    if not os.path.exists(lib_path()):
        build()
    binding.load()
    return binding


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(dom_agg_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_exports(B):
    decl = declared_functions()
    assert set(decl) == set(B.EXPORTS), decl


def test_library_exports_every_declared_symbol(B):
    lib = B.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_exported_symbols_via_nm(B):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", B.lib_path()], capture_output=True, text=True).stdout
    syms = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for name in declared_functions():
        assert name in syms, name


def test_status_strings(B):
    lib = B.load()
    for st in range(8):
        assert lib.dom_agg_status_string(st)
    assert lib.dom_agg_status_string(99) == b"unknown status"


def _plan(B, m=2, dt=None, d=1, q=1, n_inst=1, doff=None, qoff=None, flags=0, null_plan=False):
    lib = B.load()
    dt = B.F32 if dt is None else dt
    doff = np.array([0, 4] if doff is None else doff, dtype=np.int64)
    qoff = np.array([0, 3] if qoff is None else qoff, dtype=np.int64)
    h = ctypes.c_void_p()
    st = lib.dom_agg_plan(None if null_plan else ctypes.byref(h), m, dt,
                          ctypes.c_void_p(d) if d else None, ctypes.c_void_p(q) if q else None,
                          n_inst, doff.ctypes.data_as(ctypes.c_void_p), qoff.ctypes.data_as(ctypes.c_void_p),
                          flags, None)
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(m=0), "EINVAL"), (dict(m=5), "EINVAL"), (dict(null_plan=True), "EINVAL"),
    (dict(dt=3), "EUNSUPPORTED"), (dict(dt=1), "EUNSUPPORTED"), (dict(dt=9), "EINVAL"),
    (dict(n_inst=0), "EINVAL"), (dict(doff=[1, 4]), "EINVAL"), (dict(qoff=[0, -1]), "EINVAL"),
    (dict(d=0), "EINVAL"), (dict(q=0), "EINVAL"), (dict(flags=1), "EINVAL"), (dict(flags=64), "EINVAL"),
    (dict(doff=[0, 1 << 30], qoff=[0, 1 << 30]), "ETOOBIG"),
    (dict(n_inst=2, doff=[0, 3, 2], qoff=[0, 1, 3]), "EINVAL"),
    (dict(m=2, flags=0x400), "EINVAL"),          # DOM_AGG_LE(2) with m = 2
    (dict(m=1, flags=0x200), "EINVAL"),          # DOM_AGG_LE(1) with m = 1
    (dict(m=4, flags=16), "EUNSUPPORTED"),        # DOM_AGG_BASIC with m = 4
    (dict(m=4, flags=16 | 0x800), "EUNSUPPORTED"),
])
def test_plan_argument_validation(B, kw, status):
    st, _ = _plan(B, **kw)
    assert B.STATUS_NAMES[st] == status
    assert B.load().dom_agg_last_error()


def test_forward_backward_validation(B):
    lib = B.load()
    assert lib.dom_agg_forward(None, 0, B.F32, None, None, None) == B.EINVAL
    assert lib.dom_agg_backward(None, B.F32, None, None, None) == B.EINVAL
    info = B.PlanInfo()
    assert lib.dom_agg_plan_get_info(None, ctypes.byref(info)) == B.EINVAL
    lib.dom_agg_plan_destroy(None)


def test_allocator_hook_pairs(B):
    lib = B.load()
    alloc = B.ALLOC_FN(lambda n, s, c: None)
    assert lib.dom_agg_set_allocator(alloc, ctypes.cast(None, B.RELEASE_FN), None) == B.EINVAL
    assert lib.dom_agg_set_allocator(ctypes.cast(None, B.ALLOC_FN), ctypes.cast(None, B.RELEASE_FN), None) == B.OK


def _run(B, m=2, dt=None, d=1, q=1, n_inst=1, doff=None, qoff=None, op=0, wdt=None, w=1, out=1, flags=0):
    lib = B.load()
    dt = B.F32 if dt is None else dt
    wdt = B.F32 if wdt is None else wdt
    doff = np.array([0, 4] if doff is None else doff, dtype=np.int64)
    qoff = np.array([0, 3] if qoff is None else qoff, dtype=np.int64)
    p = lambda x: ctypes.c_void_p(x) if x else None  # noqa: E731
    return lib.dom_agg_run(m, dt, p(d), p(q), n_inst, doff.ctypes.data_as(ctypes.c_void_p),
                           qoff.ctypes.data_as(ctypes.c_void_p), op, wdt, p(w), p(out), flags, None)


@pytest.mark.parametrize("kw,status", [
    (dict(m=0), "EINVAL"), (dict(dt=3), "EUNSUPPORTED"), (dict(n_inst=0), "EINVAL"),
    (dict(doff=[1, 4]), "EINVAL"), (dict(d=0), "EINVAL"), (dict(flags=2), "EINVAL"), (dict(flags=4), "EINVAL"),
    (dict(op=7), "EINVAL"), (dict(wdt=9), "EINVAL"), (dict(w=0), "EINVAL"), (dict(out=0), "EINVAL"),
    (dict(doff=[0, 1 << 30], qoff=[0, 1 << 30]), "ETOOBIG"),
    (dict(m=2, flags=0x400), "EINVAL"), (dict(m=4, flags=16), "EUNSUPPORTED"),
])
def test_run_argument_validation(B, kw, status):
    st = _run(B, **kw)
    assert B.STATUS_NAMES[st] == status
    assert B.load().dom_agg_last_error()


def test_run_count_needs_no_weights_and_reports_enodev_without_device(B):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert B.STATUS_NAMES[_run(B, op=B.COUNT, w=0)] == "ENODEV"
    # nothing to write: accepted without touching a device
    assert _run(B, qoff=[0, 0], out=0) == B.OK


def test_valid_plan_without_device_reports_enodev(B):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, _ = _plan(B)
    assert B.STATUS_NAMES[st] == "ENODEV"


def test_timing_api(B):
    lib = B.load()
    assert lib.dom_agg_timing_enable(1) == B.OK
    assert B.timing_read() == {}
    assert lib.dom_agg_timing_enable(0) == B.OK


def test_python_front_end_fails_loudly_without_library(tmp_path):
    from paper_2305_16751_amd import binding
    with pytest.raises(RuntimeError, match="has not been built"):
        binding.load(str(tmp_path / "missing.so"))


def test_plan_info_layout_matches_header(B, tmp_path):
    """The ctypes mirror of dom_agg_plan_info has the C struct's size and
    field offsets (compiled from the header with the host C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    fields = [f for f, _ in B.PlanInfo._fields_]
    src = tmp_path / "layout.c"
    src.write_text(
        "#include <stddef.h>\n#include <stdio.h>\n#include \"dom_agg.h\"\n"
        "int main(void) {\n"
        "  printf(\"size %zu\\n\", sizeof(dom_agg_plan_info));\n"
        + "".join(f"  printf(\"{f} %zu\\n\", offsetof(dom_agg_plan_info, {f}));\n" for f in fields)
        + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    assert int(got["size"]) == ctypes.sizeof(B.PlanInfo)
    for f in fields:
        assert int(got[f]) == getattr(B.PlanInfo, f).offset, f


def test_no_kernel_uses_scratch_memory():
    """Every kernel keeps its per-lane state in registers and LDS: the
    compiler's resource report shows no scratch (private) memory."""
    import subprocess
    import sys
    sys.path.insert(0, ROOT)
    from paper_2305_16751_amd import build as bld
    out = os.path.join(ROOT, "_build", "scratch_check.so")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    r = subprocess.run(bld.compile_command(out, ["-Rpass-analysis=kernel-resource-usage"]),
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark:\s+(Function Name|ScratchSize \[bytes/lane\]): (\S+)", line)
        if not m:
            continue
        if m.group(1) == "Function Name":
            cur = m.group(2)
        else:
            kernels[cur] = int(m.group(2))
    assert kernels, "no resource remarks"
    assert not {k: v for k, v in kernels.items() if v}, "kernels with scratch"


def test_le_and_basic_flags_pass_validation_without_device(B):
    """Valid DOM_AGG_LE / DOM_AGG_BASIC flags get past validation: with no
    device the call then reports ENODEV, not EINVAL."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    for m, flags in ((2, B.LE(0) | B.LE(1)), (3, B.BASIC | B.LE(2)), (1, B.BASIC)):
        st, _ = _plan(B, m=m, flags=flags)
        assert B.STATUS_NAMES[st] == "ENODEV", (m, flags)
