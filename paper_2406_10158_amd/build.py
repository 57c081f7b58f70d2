"""Build the engine's shared library (libcc.so) for gfx950 with hipcc.

Usage: python -m paper_2406_10158_amd.build
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcc.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("txn_occ.hip", "txn_2pl.hip", "txn_2plwd.hip", "txn_to.hip", "txn_mvcc.hip", "txn_tictoc.hip", "gacco.hip",
            "gacco_exec.hip", "gputx.hip", "index.hip", "ingest.hip", "kernels.hip", "roofline.hip", "static_run.hip", "api.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled in all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include")]
# The OCC sources hold the hot-row engine, whose LDS atomics are issued by one
# lane that owns the row (or are already aggregated per wavefront by hand): the
# compiler's wavefront aggregation of atomics would only lengthen its critical
# sections.
EXTRA_FLAGS = {"txn_occ.hip": ["-Xarch_device", "-mllvm=-amdgpu-atomic-optimizer-strategy=None"]}


def build(verbose: bool = False) -> str:
    """Compile every source and link libcc.so in-tree; always rebuilds."""
    tmpdir = os.path.join(PKG, "_build")
    os.makedirs(tmpdir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
        cmd = [HIPCC, f"--offload-arch={ARCH}", *COMMON, "-c", src, "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = DEVICE_FLAGS + EXTRA_FLAGS.get(os.path.basename(src), [])
        cmds.append((src, cmd))
        objs.append(obj)

    def compile_one(item):
        src, cmd = item
        if verbose:
            print(" ".join(cmd), flush=True)
        return src, subprocess.run(cmd, capture_output=True, text=True)

    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as pool:
        for src, r in pool.map(compile_one, cmds):
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc failed on {src}")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libcc.so failed")
    os.replace(tmp, LIB)
    shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
