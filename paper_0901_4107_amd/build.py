"""Build libmm.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBMM = os.path.join(HERE, "libmm.so")
LIBVOR = os.path.join(HERE, "inputs", "libvoronoi.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: some of their forms have been seen
    # to give wrong results without an error on this hardware
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core accumulators in ordinary VGPRs: the fused network then
    # shares the register file with the flux code instead of adding AGPRs
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    # single precision only (the double path compiles to the same code):
    # float division and square root by the hardware reciprocal and root
    # (about 1 ulp) instead of correctly rounded sequences, float denormals
    # flushed. The float path's error budget is the 1e-6 L1 of the mixed
    # form, far above these roundings; its states never approach 1e-38.
    "-fno-hip-fp32-correctly-rounded-divide-sqrt", "-fgpu-flush-denormals-to-zero",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def source_hash() -> str:
    """Short hash of the code of the kernel sources (comments and layout
    whitespace removed) and the flags libmm is built from; tags
    measurements taken from a particular build of the kernels."""
    import hashlib
    import re

    def code(text: str) -> str:
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        return " ".join(text.split())

    h = hashlib.sha256(" ".join(HIPCC_FLAGS).encode())
    files = [os.path.join(CSRC, name) for name in sorted(os.listdir(CSRC))]
    for path in files + [os.path.join(ROOT, "include", "mm.h")]:
        with open(path) as fh:
            h.update(os.path.basename(path).encode())
            h.update(code(fh.read()).encode())
    return h.hexdigest()[:16]


def build_libmm(extra=()) -> str:
    src = os.path.join(CSRC, "mm.hip")
    cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-o", LIBMM + ".tmp", src]
    subprocess.check_call(cmd)
    os.replace(LIBMM + ".tmp", LIBMM)
    return LIBMM


def build_voronoi() -> str:
    src = os.path.join(HERE, "inputs", "voronoi.cpp")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", LIBVOR + ".tmp", src])
    os.replace(LIBVOR + ".tmp", LIBVOR)
    return LIBVOR


def build_all() -> None:
    build_voronoi()
    build_libmm()


if __name__ == "__main__":
    build_all()
