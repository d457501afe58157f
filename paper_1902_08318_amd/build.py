"""Build step for the HIP library (gfx950).

Compiles csrc/jsidx.hip, csrc/jsidx_noalloc.hip, csrc/jsidx_scopes.hip and csrc/jsidx_tape.hip with hipcc into libjsidx.so
next to this file.  The
build runs on a machine without a GPU: hipcc cross-compiles for gfx950.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjsidx.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
    # packed FP32 instructions are not wanted anywhere in this code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build_library(verbose: bool = False) -> str:
    """Compile the HIP library; returns the path of libjsidx.so."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *HIP_FLAGS, "-o", tmp, os.path.join(CSRC, "jsidx.hip"), os.path.join(CSRC, "jsidx_noalloc.hip"),
           os.path.join(CSRC, "jsidx_scopes.hip"), os.path.join(CSRC, "jsidx_tape.hip")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "'-packed-fp32-ops' is not a recognized feature"
    msgs = [l for l in (res.stdout + res.stderr).splitlines() if noise not in l]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
