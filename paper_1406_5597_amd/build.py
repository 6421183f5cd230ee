"""Build libfft3d.so in-tree with hipcc for gfx950.

    python -m paper_1406_5597_amd.build

Compiles the HIP kernels and the host C++ (plan, C ABI) in parallel into
``_build/`` next to this file and links ``libfft3d.so`` beside it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfft3d.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Device code: gfx950 only; no contraction beyond the explicit fma calls in the
# sources (so rounding is fixed by the source); packed FP32 instructions off.
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
                "-I" + INCLUDE]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "--offload-arch=" + ARCH, "--cuda-host-only", "-I" + INCLUDE]

# Longest compiles first (they bound the wall time; the pool runs one per core).
SOURCES = [
    ("fft3d_kern_f32_odd.hip", DEVICE_FLAGS),
    ("fft3d_kern_f64_odd.hip", DEVICE_FLAGS),
    ("fft3d_kern_f32.hip", DEVICE_FLAGS),
    ("fft3d_kern_f64.hip", DEVICE_FLAGS),
    ("fft3d_pruned_f32_odd.hip", DEVICE_FLAGS),
    ("fft3d_pruned_f64_odd.hip", DEVICE_FLAGS),
    ("fft3d_pruned_f32.hip", DEVICE_FLAGS),
    ("fft3d_pruned_f64.hip", DEVICE_FLAGS),
    ("fft3d_batch.hip", DEVICE_FLAGS),
    ("fft3d_level.hip", DEVICE_FLAGS),
    ("fft3d_coop_f32.hip", DEVICE_FLAGS),
    ("fft3d_coop_f64.hip", DEVICE_FLAGS),
    ("fft3d_batch_host.cpp", HOST_FLAGS),
    ("fft3d_server.cpp", HOST_FLAGS),
    ("fft3d_plan.cpp", HOST_FLAGS),
    ("fft3d_tune.cpp", HOST_FLAGS),
    ("fft3d_dispatch.cpp", HOST_FLAGS),
    ("fft3d_abi.cpp", HOST_FLAGS),
]


def _compile(src: str, flags) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + list(flags) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), err))
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    workers = max(1, min(len(SOURCES), os.cpu_count() or 1, int(os.environ.get("MAX_JOBS", "64"))))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
