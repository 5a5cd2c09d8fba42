"""Build the gfx950 shared library libebicg.so in-tree with hipcc.

Usage: python -m paper_0911_2285_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libebicg.so")
ARCH = "gfx950"

# device code: no packed-FP32 instructions (some of their forms gave wrong results on MI355X);
# matrix instructions with their accumulators in ordinary VGPRs: left to its heuristics the
# compiler kept the accumulators of the tiled products in VGPRs but issued the AGPR form,
# copying 8 registers in and out around every pair of MFMAs and draining the pipeline between them
HIP_FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wno-unused-result",
]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fcx-limited-range"]

SOURCES = [
    ("kernels.hip", "hip"),
    ("api.hip", "hip"),
    ("tsmm.hip", "hip"),
    ("batch.hip", "hip"),
    ("eo.hip", "hip"),
    ("winrestart.hip", "hip"),
    ("hostla.cpp", "host"),
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source and link libebicg.so; returns its path."""
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(item):
        src, kind = item
        obj = os.path.join(objdir, src + ".o")
        flags = HIP_FLAGS if kind == "hip" else HOST_FLAGS
        cmd = [hipcc, *flags, "-I", INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile {src} failed:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
