"""Build librpod.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librpod.so")
SOURCES = ["stream_kernels.hip", "stream16_kernels.hip", "stream_e6_kernels.hip", "small_kernels.hip", "center_kernels.hip", "energy_kernels.hip", "recon_kernels.hip",
           "warm_kernels.hip", "rpod_abi.cpp", "warm_abi.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose=True):
    """Compile every source into librpod.so (always rebuilds)."""
    from concurrent.futures import ThreadPoolExecutor
    jobs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC, "-x", "hip", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((cmd, obj))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "6"))))
    with ThreadPoolExecutor(workers) as ex:
        for fut in [ex.submit(subprocess.run, cmd, check=True) for cmd, _ in jobs]:
            fut.result()
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
