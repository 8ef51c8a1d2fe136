"""Build libqtt.so (HIP, gfx950) in-tree with hipcc.

Every ``csrc/*.hip`` translation unit is compiled on its own (in parallel)
and the objects are linked into ``libqtt.so``.

Usage: python -m paper_1511_06029_amd.build_lib
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libqtt.so")
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; set HIPCC or install ROCm")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln)
    return res.returncode, errs


def build(verbose=True, jobs=None):
    """Compile the HIP sources into LIB; returns its path.  Always rebuilds."""
    os.makedirs(OBJDIR, exist_ok=True)
    flags = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             # packed FP32 instructions are kept out of the device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC]
    srcs = sources()
    objs = [os.path.join(OBJDIR, os.path.basename(s)[:-4] + ".o") for s in srcs]
    cmds = [[hipcc()] + flags + ["-c", "-o", o, s] for s, o in zip(srcs, objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    failed = [(c[-1], rc, e) for c, (rc, e) in zip(cmds, results) if rc != 0]
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(f"{s} ({rc}):\n{e}" for s, rc, e in failed))
    if verbose:
        for _, e in results:
            if e.strip():
                print(e, file=sys.stderr)
    tmp = LIB + ".tmp"
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    rc, errs = _run(link)
    if rc != 0:
        raise RuntimeError(f"link failed ({rc}):\n{errs}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
