"""Build the HIP library (gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libqnsch_hip.so")
SOURCES = ["qnsch_lib.hip"]
ARCH = "gfx950"

# Packed FP32 instructions are switched off for all device code.
HIPFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=fast",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


# the device code: the kernels and the functions they inline (the host
# library around them does not change what a kernel reads and writes)
DEVICE_SOURCES = ["qnsch_dev.hpp", "qnsch_lin.hpp", "qnsch_kern.hpp", "qnsch_mxk.hpp"]


def device_source_hash():
    """short hash of the device code; profile summaries taken on other
    device code are stale"""
    import hashlib
    h = hashlib.sha256()
    for f in DEVICE_SOURCES:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def build(verbose=False):
    objs = []
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(bdir, os.path.splitext(s)[0] + ".o")
        cmd = ["hipcc", "-c", src, "-o", obj, "-I", os.path.join(ROOT, "include"), "-I", CSRC] + HIPFLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
