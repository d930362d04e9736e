"""Build the gfx950 shared library (the C ABI of include/mrtfd.h) in-tree.

    python -m paper_1305_4736_amd.build

compiles paper_1305_4736_amd/csrc/mrtfd.hip and mrtfd_batch.hip with hipcc for gfx950 into
paper_1305_4736_amd/libmrtfd.so.  Packed FP32 instructions are disabled for
the device code (``-Xclang -target-feature -Xclang -packed-fp32-ops``).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", n) for n in ("mrtfd.hip", "mrtfd_batch.hip")]
LIB = os.path.join(HERE, "libmrtfd.so")
HEADERS = [os.path.join(HERE, "csrc", n) for n in ("mrtfd_device.h", "mrtfd_consts.h")] + [
    os.path.join(ROOT, "include", "mrtfd.h")]

ARCH = os.environ.get("MRTFD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # a * b + c is fused only within one source expression, so every
         # kernel that shares a device function rounds it the same way
         "-ffp-contract=on",
         # device code flushes denormals (FP32 and FP64), which lets the
         # limiter scale by an instruction's output modifier; the host part
         # keeps the default
         "-Xarch_device", "-fdenormal-fp-math=preserve-sign",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, *FLAGS, "-o", tmp, *[s for s in SRCS if os.path.exists(s)]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
    sys.exit(0)
