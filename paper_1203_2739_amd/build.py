"""Build libspx.so in-tree for gfx950.

Device code is compiled by hipcc; packed FP32 instructions are disabled
(``-packed-fp32-ops``) and binary64 atomics use the hardware instruction
(``-munsafe-fp-atomics``).  Host-only sources are compiled by the same clang
as host C++.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libspx.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
ARCH = "gfx950"

DEVICE_SOURCES = ["kernels.hip", "mlp.hip"]
HOST_HIP_SOURCES = ["api.cpp", "lowp.cpp", "batch.cpp", "selector.cpp", "tune.cpp", "orderings.cpp"]
HOST_SOURCES = ["partition.cpp", "plan.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function"]
DEVICE_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops", "-munsafe-fp-atomics", "-fno-gpu-flush-denormals-to-zero"]


def _extra_sources():
    """Sources added by later components (listed in csrc/SOURCES if present)."""
    path = os.path.join(CSRC, "SOURCES")
    dev, host = [], []
    if os.path.exists(path):
        for line in open(path):
            line = line.split("#")[0].strip()
            if not line:
                continue
            (dev if line.endswith(".hip") else host).append(line)
    return dev, host


def _cmd_for(src: str, obj: str):
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        return [HIPCC, "-x", "hip", *COMMON, *DEVICE_FLAGS, "-c", path, "-o", obj]
    if src in HOST_HIP_SOURCES:
        return [CLANGXX, *COMMON, "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-c", path,
                "-o", obj]
    return [CLANGXX, *COMMON, "-c", path, "-o", obj]


def build(verbose: bool = False) -> str:
    """Compile every source and link libspx.so; returns the library path."""
    os.makedirs(OUT_DIR, exist_ok=True)
    dev_extra, host_extra = _extra_sources()
    sources = DEVICE_SOURCES + dev_extra + HOST_HIP_SOURCES + HOST_SOURCES + host_extra
    jobs = []
    for src in sources:
        obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
        jobs.append((src, obj, _cmd_for(src, obj)))

    def run(job):
        src, obj, cmd = job
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
        if r.stderr.strip() and verbose:
            print(r.stderr, file=sys.stderr)
        return obj

    workers = min(len(jobs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        objs = list(ex.map(run, jobs))
    tmp = LIB + ".tmp"
    link = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libspx.so failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
