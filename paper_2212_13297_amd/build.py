"""Compile the HIP library in-tree for gfx950.

Produces ``paper_2212_13297_amd/libhercules_hip.so`` from ``csrc/`` with
hipcc (one compiler process per source file, then one link).  Every HIP
translation unit is built with packed-FP32 instruction generation disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhercules_hip.so")
SOURCES = ["csrc/hs_build.hip", "csrc/hs_query.hip", "csrc/hs_filter.hip", "csrc/hs_refine.hip", "csrc/hs_scan.hip",
           "csrc/hs_precision.hip", "csrc/hs_static.hip", "csrc/hs_partition.hip", "csrc/hs_api.cpp", "csrc/hs_server.cpp"]
ARCH = os.environ.get("HS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel (one hipcc per file),
    then link the shared library."""
    import concurrent.futures as cf
    import tempfile
    flags = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory(prefix="hs_build_") as tmpdir:
        objs = []
        cmds = []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            objs.append(obj)
            cmds.append([hipcc()] + flags + ["-c", os.path.join(HERE, src), "-o", obj])

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)

        workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
        with cf.ThreadPoolExecutor(workers) as ex:
            list(ex.map(run, cmds))
        tmp = LIB + ".tmp"
        link = [hipcc(), f"--offload-arch={ARCH}", "-fPIC", "-shared", "-o", tmp] + objs
        run(link)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
