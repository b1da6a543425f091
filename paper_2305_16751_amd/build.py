"""Builds the HIP library libdom_agg.so in-tree for gfx950.

    python -m paper_2305_16751_amd.build

All kernels and the C-ABI live in csrc/dom_agg.hip (one translation unit);
include/dom_agg.h is the public header.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_NAME = "libdom_agg.so"
SOURCES = [os.path.join(PKG, "csrc", "dom_agg.hip")]
HEADERS_DIRS = [os.path.join(ROOT, "include"), os.path.join(PKG, "csrc")]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def lib_path() -> str:
    return os.path.join(PKG, LIB_NAME)


def compile_command(out: str, extra: list[str] | None = None, root: str | None = None) -> list[str]:
    """hipcc command line; root: a copy of the sources made by snapshot()
    (default: the tree itself)."""
    cmd = [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
           # no packed fp32 instructions in any kernel
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
    inc, srcs = HEADERS_DIRS, SOURCES
    if root is not None:
        inc = [os.path.join(root, "include"), os.path.join(root, "csrc")]
        srcs = [os.path.join(root, "csrc", os.path.basename(f)) for f in SOURCES]
    for d in inc:
        cmd += ["-I", d]
    cmd += extra or []
    cmd += ["-o", out] + srcs
    return cmd


def snapshot(dst: str) -> str:
    """Copies the sources and headers into dst.  hipcc reads the sources once
    for the device pass and again, minutes later, for the host pass; compiling
    a copy keeps both passes on one version of every file (a struct that
    changed in between would otherwise be laid out differently on the two
    sides of a kernel launch)."""
    shutil.copytree(HEADERS_DIRS[0], os.path.join(dst, "include"))
    shutil.copytree(HEADERS_DIRS[1], os.path.join(dst, "csrc"),
                    ignore=shutil.ignore_patterns("*.so", "*.so.tmp*"))
    return dst


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    out = lib_path()
    tmp = out + ".tmp%d" % os.getpid()
    with tempfile.TemporaryDirectory(prefix="dom_agg_src_") as d:
        cmd = compile_command(tmp, extra, root=snapshot(d))
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the device feature above; that warning is harmless
    msgs = [ln for ln in (res.stderr or "").splitlines() if "packed-fp32-ops" not in ln]
    if res.returncode != 0:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
