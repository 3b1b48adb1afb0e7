"""Build ``libkt.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
SOURCES = [os.path.join(_HERE, "csrc", "kt_main.hip")]
DEPENDS = SOURCES + [os.path.join(_HERE, "csrc", "kt_device.hpp"),
                     os.path.join(_ROOT, "include", "kt.h")]
LIB = os.path.join(_HERE, "libkt.so")

HIPCC_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
               # a*b + c is fused where the source writes it, never across statements: the
               # rounding then does not depend on how a device function is inlined, so the
               # batched kernels reproduce the single-event kernels bit for bit
               "-ffp-contract=on",
               # no packed FP32 instructions in any kernel
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I" + os.path.join(_ROOT, "include"), "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
