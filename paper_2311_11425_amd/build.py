"""Build the gfx950 HIP library libhevi.so in-tree (cross-compiles without a GPU)."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhevi.so")
SOURCES = ["hevi_kernels.hip", "hevi_kernels3c.hip", "hevi_ps.hip", "hevi_group.hip",
           "hevi_noalloc.hip", "hevi_api.cpp",
           "hevi_group_api.cpp", "hevi_serve.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # no packed-FP32 instructions in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        "-Wall", "-Wno-unused-function",
    ]


def _stale(obj, src):
    """True if obj is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    deps = [src] + glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(ROOT, "include", "hevi.h")]
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, only_changed: bool = False) -> str:
    """Compile every source for gfx950 (in parallel) and link libhevi.so.
    only_changed skips objects that are newer than their inputs."""
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    jobs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src + ".o")
        path = os.path.join(CSRC, src)
        objs.append(obj)
        if only_changed and not _stale(obj, path):
            continue
        jobs.append([HIPCC] + flags() + ["-x", "hip", "-c", path, "-o", obj])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    with ThreadPoolExecutor(max_workers=max(1, min(len(jobs), 8))) as ex:
        for f in [ex.submit(run, c) for c in jobs]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, only_changed="--changed" in sys.argv))
