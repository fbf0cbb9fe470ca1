"""Compile libpcfgsmc.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpcfgsmc.so")
SOURCES = ["kernels.hip", "capi.hip"]
HEADERS = ["devmath.hpp", "models.hpp", "engine.hpp", "launch.hpp", "program.hpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # one rounding per written operation: no contraction into FMAs, no fast-math
    "-ffp-contract=off", "-fno-fast-math",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def command(out: str = LIB) -> list[str]:
    return [hipcc(), *HIPCC_FLAGS, "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
            "-o", out, *[os.path.join(CSRC, s) for s in SOURCES]]


def build(verbose: bool = False) -> str:
    """Always recompiles; writes the library atomically."""
    tmp = f"{LIB}.{os.getpid()}.tmp"  # per process: concurrent builds do not collide
    r = subprocess.run(command(tmp), capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr[-4000:])
    if verbose and r.stderr:
        print(r.stderr)
    os.replace(tmp, LIB)
    return LIB


def sources_newer_than_lib() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    files = [os.path.join(CSRC, f) for f in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "pcfgsmc.h")]
    return any(os.path.getmtime(f) > t for f in files)


if __name__ == "__main__":
    print(build(verbose=True))
