"""Build step for the HIP library (gfx950)."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libslpic.so")
SOURCES = [os.path.join(CSRC, "slpic_capi.cpp"),
           os.path.join(CSRC, "slpic_kernels.hip")]
HEADERS = [os.path.join(CSRC, "slpic_internal.hpp"),
           os.path.join(os.path.dirname(HERE), "include", "slpic.h")]


def hipcc_command(out=LIB):
    return ["hipcc", "-shared", "-fPIC", "-O3", "--offload-arch=gfx950",
            "-std=c++17", "-Wall",
            # packed FP32 instructions stay off: plain float code only
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-o", out] + SOURCES


def build(verbose=False):
    cmd = hipcc_command()
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = ("packed-fp32-ops", "warning: unknown target feature")
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines()
            if ln.strip() and not any(n in ln for n in noise)]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)
