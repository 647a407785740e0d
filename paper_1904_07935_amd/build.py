"""Build the HIP library in-tree with hipcc for gfx950.

Compiles every source under csrc/ to an object in _build/ and links
``libplnmf.so`` next to this file.  Always rebuilds (used by
``__graft_entry__.build()``); ``python -m paper_1904_07935_amd.build`` runs it
by hand.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libplnmf.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


# The W kernel keeps a 32-column tile per row in registers, and the GEMM's
# epilogue walks its accumulator blocks: both loops must unroll fully (static
# register indices, no private-memory copy), past the default size limit.
_FULL_UNROLL = ["-mllvm", "-pragma-unroll-threshold=1000000"]
EXTRA = {"hals.hip": _FULL_UNROLL, "gemm.hip": _FULL_UNROLL}


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src):
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
    return obj, msgs


CPU_SRC = os.path.join(HERE, "cpu", "plnmf_cpu.cpp")
CPU_LIB = os.path.join(HERE, "libplnmf_cpu.so")


def build_cpu(verbose=False):
    """The PL-NMF-cpu baseline (FP64, OpenMP): a host library of its own."""
    tmp = CPU_LIB + ".tmp"
    cmd = [os.environ.get("CXX", "g++"), "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           "-std=c++17", "-Wall", CPU_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("g++ failed on plnmf_cpu.cpp:\n" + r.stdout + r.stderr)
    if verbose and (r.stdout + r.stderr).strip():
        print(r.stdout + r.stderr, file=sys.stderr)
    shutil.move(tmp, CPU_LIB)
    return CPU_LIB


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(_compile, sources()))
    objs = []
    for obj, msgs in results:
        objs.append(obj)
        if verbose and msgs.strip():
            print(msgs, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    shutil.move(tmp, LIB)
    build_cpu(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
