"""Build libbf.so in-tree for gfx950 with hipcc.

Every call recompiles.  The library is written next to this file so that it
travels with the source tree; nothing is installed.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbf.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are switched off in every HIP translation unit.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]

# extra device flags for diagnostics, e.g. BF_HIPCC_EXTRA="-Rpass-analysis=kernel-resource-usage"
EXTRA = os.environ.get("BF_HIPCC_EXTRA", "").split()

SOURCES = [
    ("bf_tables.cpp", False),
    ("bf_kernels.hip", True),
    ("bf_toeplitz.hip", True),
    ("bf_api.hip", True),
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    """Compile the translation units concurrently (at most MAX_JOBS or the CPU
    count at once), then link."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for name, is_hip in SOURCES:
        src = os.path.join(CSRC, name)
        if not os.path.exists(src):
            raise FileNotFoundError(f"translation unit {src} is missing")
        obj = os.path.join(BUILD, name + ".o")
        cmd = [HIPCC, "-c"] + (["-x", "hip"] if is_hip else []) + [src, "-o", obj] + COMMON
        if is_hip:
            cmd += DEVICE_FLAGS + EXTRA
        jobs.append((cmd, obj))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        for f in [pool.submit(_run, cmd, verbose) for cmd, _ in jobs]:
            f.result()  # re-raises a failed compile
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
