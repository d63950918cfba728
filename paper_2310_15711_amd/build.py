"""Build libhc.so (HIP for gfx950 + host C++) in-tree with hipcc.

Usage: python -m paper_2310_15711_amd.build [--force]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libhc.so")
LOADGEN = os.path.join(PKG, "libhc_loadgen.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]
# no packed fp32 instructions in device code (there is no fp32 math on this
# path, the flag only rules them out)
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

SOURCES = [
    "hc_preprocess.cpp",
    "hc_runtime.hip",
    "hc_search.hip",
    "hc_batched.hip",
    "hc_serve.cpp",
    "hc_autotune.cpp",
    "hc_preprocess_device.hip",
]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, *COMMON, *DEVICE, "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, "-c", path, "-o", obj]
    subprocess.check_call(cmd)
    return obj


def build(force: bool = True, jobs: int | None = None) -> str:
    """Compile every source and link libhc.so. Always recompiles when force."""
    os.makedirs(OBJ, exist_ok=True)
    headers = [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    headers.append(os.path.join(INCLUDE, "hc.h"))
    newest_header = max(os.path.getmtime(h) for h in headers)

    def stale(src):
        obj = os.path.join(OBJ, src + ".o")
        if force or not os.path.exists(obj):
            return True
        t = os.path.getmtime(obj)
        return t < os.path.getmtime(os.path.join(CSRC, src)) or t < newest_header

    todo = [s for s in SOURCES if stale(s)]
    with cf.ThreadPoolExecutor(max_workers=jobs or min(8, os.cpu_count() or 4)) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(OBJ, s + ".o") for s in SOURCES]
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp,
                           "-lpthread"])
    os.replace(tmp, LIB)
    # the benchmark's load generator: a small host library on top of libhc
    gen_tmp = LOADGEN + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", "-I", INCLUDE,
                           os.path.join(CSRC, "hc_loadgen.cpp"), "-o", gen_tmp, "-L", PKG, "-lhc",
                           "-Wl,-rpath,$ORIGIN", "-lpthread"])
    os.replace(gen_tmp, LOADGEN)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv)
    print(LIB)
