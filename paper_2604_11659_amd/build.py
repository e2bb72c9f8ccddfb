"""Builds libfhe_spmspm.so (HIP, gfx950) in-tree from csrc/ with hipcc.

Usage: python -m paper_2604_11659_amd.build [--jobs N] [--sanitize]

--sanitize builds libfhe_spmspm_san.so instead: the same sources with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only (device code is built as usual), for CPU runs of
the host-only entry points under a preloaded clang ASan runtime (see host_asan_runtime()).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfhe_spmspm.so")
OBJ_SAN = os.path.join(HERE, "_build_san")
LIB_SAN = os.path.join(HERE, "libfhe_spmspm_san.so")
# host-only sanitizers: every -fsanitize sits behind -Xarch_host, so no device code is instrumented
SAN_FLAGS = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
             "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer").split()
SAN_LINK = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -shared-libasan".split()
SOURCES = ["kernels.hip", "runtime.cpp", "host_math.cpp", "ckks.cpp", "spmspm.cpp", "server.cpp", "tune.cpp", "noalloc.hip", "capi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("FHE_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-result", "-Wno-pass-failed",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(OBJ_SAN if sanitize else OBJ, os.path.splitext(src)[0] + ".o")
    extra = [*SAN_FLAGS, "-g"] if sanitize else []
    cmd = [HIPCC, "-x", "hip", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, sanitize: bool = False) -> str:
    os.makedirs(OBJ_SAN if sanitize else OBJ, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize), SOURCES))
    lib = LIB_SAN if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread",
           *(SAN_LINK if sanitize else [])]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


def host_asan_runtime() -> str:
    """The clang ASan runtime that a process loading the sanitized library must preload."""
    r = subprocess.run([os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("clang ASan runtime not found")
    return path


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--sanitize", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.sanitize))
    sys.exit(0)
