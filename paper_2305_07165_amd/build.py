"""Builds libfgt.so (host plan + gfx950 kernels) in the package directory.

Host C++ (plan, tables) is compiled with g++; the HIP sources with hipcc for
gfx950 only.  Packed FP32 instructions are disabled for all device code.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfgt.so")

HOST_SRC = ["plan.cpp", "tables.cpp", "output_host.cpp", "point_host.cpp"]
HIP_SRC = ["persist.hip", "kernels.hip", "kernels_fast.hip", "api.hip", "serve.hip", "batch.hip", "output.hip", "point.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
              "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def _stale(obj: str, src: str) -> bool:
    """True when obj is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(d, f) for d in (CSRC, os.path.join(ROOT, "include"))
                    for f in os.listdir(d) if f.endswith(".h")]
    return any(os.path.getmtime(x) > t for x in deps)


def build(verbose: bool = True, incremental: bool = False) -> str:
    """Compiles every source (incremental=True: only objects older than their
    source or a header) and links libfgt.so and the ceilings probe."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in HOST_SRC:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], obj, src))
    for src in HIP_SRC:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], obj, src))
    todo = [cmd for cmd, obj, src in jobs
            if not incremental or _stale(obj, os.path.join(CSRC, src))]
    # independent translation units compile in parallel
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(_run, cmd) for cmd in todo]:
            f.result()
    objs = [obj for _, obj, _ in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    # roofline ceilings probe (matrix cores, vector FMA, copy), a separate program
    exe = os.path.join(HERE, "fgt_ceilings")
    _run([HIPCC, "--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-o", exe + ".tmp", os.path.join(CSRC, "ceilings.hip")])
    os.replace(exe + ".tmp", exe)
    return LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
    sys.exit(0)
