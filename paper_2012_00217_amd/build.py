"""Compile libmbl.so (all HIP sources under csrc/) for gfx950 with hipcc.

Run as ``python -m paper_2012_00217_amd.build``.  Objects go to ``_build/``
at the repository root; the shared library is written next to this file.
A measurement variant of the kernels (a compile-time switch of the sources) is
built with extra flags into another file, e.g.

    MBL_HIPCC_FLAGS=-DMBL_CG_NT_LOAD=1 MBL_BUILD_OUT=/tmp/nt/libmbl.so \
        python -m paper_2012_00217_amd.build

and loaded instead of the default library with MBL_LIBRARY=/tmp/nt/libmbl.so.
"""

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmbl.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MBL_OFFLOAD_ARCH", "gfx950")
# MBL_HIPCC_FLAGS: extra compiler flags, e.g. "-DMBL_CG_NT_LOAD=1" to build a
# variant of the kernels for a measurement (MBL_LIBRARY then selects it).
EXTRA = os.environ.get("MBL_HIPCC_FLAGS", "").split()
OUT = os.environ.get("MBL_BUILD_OUT", OUT)
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are disabled for every device function
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
] + EXTRA


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    tag = "" if not EXTRA else "." + hashlib.sha1(" ".join(EXTRA).encode()).hexdigest()[:8]
    obj = os.path.join(BUILD, os.path.basename(src) + tag + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")), 16)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile, srcs))
    os.makedirs(os.path.dirname(os.path.abspath(OUT)), exist_ok=True)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
