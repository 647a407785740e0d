"""Sanitizer build of the host code (CPU only; never shipped to a GPU).

Builds libplnmf.so with AddressSanitizer and UndefinedBehaviorSanitizer on
the host side of every source (device code is compiled unchanged) and
libplnmf_cpu.so with both sanitizers, into _build_asan/, then runs the CPU
tests that exercise them (the C-ABI argument checks and workspace carving,
and PL-NMF-cpu against the oracle) with the sanitizer runtime preloaded:

    python -m paper_1904_07935_amd.build_sanitize
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

from . import build as b

OUT = os.path.join(b.HERE, "_build_asan")
SAN = "-fsanitize=address,undefined"


def _compile(src):
    obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    cmd = ([b.HIPCC] + b.COMMON + b.EXTRA.get(src, []) +
           ["-Xarch_host", SAN, "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g",
            "-c", os.path.join(b.CSRC, src), "-o", obj])
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}{r.stderr}")
    return obj


def asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang's ASan runtime not found")
    return hits[-1]


def main():
    os.makedirs(OUT, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, b.sources()))
    lib = os.path.join(OUT, "libplnmf.so")
    r = subprocess.run([b.HIPCC, "-shared", "-fPIC", f"--offload-arch={b.ARCH}", "-Xarch_host", SAN,
                        "-o", lib] + objs, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    cpu_lib = os.path.join(OUT, "libplnmf_cpu.so")
    # clang++ from the same toolchain, so that both libraries use one ASan runtime
    clang = os.path.join(os.path.dirname(b.HIPCC), "..", "llvm", "bin", "clang++")
    omp_dir = os.path.join(os.path.dirname(b.HIPCC), "..", "llvm", "lib")
    r = subprocess.run([clang, "-O1", "-g", "-fno-omit-frame-pointer", SAN, "-fopenmp", "-fPIC",
                        "-shared", "-std=c++17", f"-L{omp_dir}", f"-Wl,-rpath,{omp_dir}", b.CPU_SRC,
                        "-o", cpu_lib], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("g++ failed:\n" + r.stdout + r.stderr)
    env = dict(os.environ, PLNMF_LIB=lib, PLNMF_CPU_LIB=cpu_lib,
               LD_PRELOAD=asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    root = os.path.dirname(b.HERE)
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
           "tests/test_abi.py", "tests/test_cpu_plnmf.py"]
    return subprocess.run(cmd, cwd=root, env=env).returncode


if __name__ == "__main__":
    sys.exit(main())
