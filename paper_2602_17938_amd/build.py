"""Build liblacosmic.so in place for gfx950.

Steps: generate the selection-network header, then one hipcc invocation over
the HIP sources.  Device code is compiled with -ffp-contract=off (no FMA
contraction) and HIP's default correctly-rounded binary32 division and square
root, so the kernels evaluate the same IEEE expression trees as a plain CPU
evaluation of the method.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN_DIR = os.path.join(ROOT, "_build", "gen")
LIB = os.path.join(HERE, "liblacosmic.so")

SOURCES = ["lacosmic_kernels.hip", "lacosmic_noalloc.hip", "lacosmic_capi.cpp",
           "lacosmic_batch.cpp", "lacosmic_server.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    # packed FP32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def generate():
    os.makedirs(GEN_DIR, exist_ok=True)
    out = os.path.join(GEN_DIR, "median_net.gen.h")
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_median_net.py"), out])
    return out


def build(verbose=False, extra_flags=()):
    generate()
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, *extra_flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-I", GEN_DIR, *srcs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
