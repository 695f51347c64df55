"""Build libpamd.so (HIP, gfx950) in-tree with hipcc, and its bounds-checked
variant libpamd_check.so (the resampling kernels compiled with
PAMD_BOUNDS_CHECK: every scan offset and gather source index is verified on
the device and reported as PAMD_ERR_INTERNAL; otherwise the same objects).

    python -m paper_1806_06016_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpamd.so")
CHECK_LIB = os.path.join(HERE, "libpamd_check.so")
CHECKED_SOURCES = ["resample.hip"]   # the sources that hold bounds checks
SOURCES = ["md_kernel.hip", "resample.hip", "runtime.hip", "nn_kernel.hip", "nn_runtime.hip", "calib.hip", "analysis.cpp"]
ARCH = os.environ.get("PAMD_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
    # packed FP32 VALU instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compile every source (always) and link libpamd.so and libpamd_check.so.
    Returns the path of libpamd.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    hipcc = _hipcc()

    def compile_one(job):
        src, checked = job
        stem = os.path.splitext(src)[0] + ("_check" if checked else "")
        obj = os.path.join(objdir, stem + ".o")
        cmd = [hipcc, *FLAGS, *extra_flags, *(["-DPAMD_BOUNDS_CHECK"] if checked else []), "-c",
               os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    jobs = [(src, False) for src in SOURCES] + [(src, True) for src in CHECKED_SOURCES]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        objs = dict(zip(jobs, ex.map(compile_one, jobs)))
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    for lib, checked in ((LIB, False), (CHECK_LIB, True)):
        parts = [objs[(src, checked and src in CHECKED_SOURCES)] for src in SOURCES]
        tmp = lib + ".tmp"
        # roctx: named ranges of the C-ABI calls in rocprofv3 marker traces
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *parts, "-o", tmp, f"-L{rocm}/lib",
               "-lrocprofiler-sdk-roctx"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
