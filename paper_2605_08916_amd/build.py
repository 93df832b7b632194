"""Build the HIP library libdr.so for gfx950 in-tree (hipcc cross-compiles
without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdr.so")
SOURCES = [os.path.join(CSRC, "dr_lib.hip"), os.path.join(CSRC, "bvh_build.cpp")]
DEPS = SOURCES + [os.path.join(CSRC, h) for h in ("dr_device.h", "dr_adjoint.h", "dr_chain.h", "dr_machine.h")] + [
    os.path.join(ROOT, "include", "dr.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    # fuse multiply-add only within one source expression: the same arithmetic
    # then compiles to the same operations wherever it is inlined, so the
    # kernels that evaluate a path in different ways agree bit for bit
    "-ffp-contract=on",
    # keep private arrays out of LDS: the traversal stack owns the dynamic LDS
    "-mllvm", "-disable-promote-alloca-to-lds",
    # packed FP32 instructions stay off (they are not needed and some forms
    # have given wrong results on this hardware).  The device pass honours the
    # feature (a float2 multiply-add compiles to v_pk_fma_f32 without it and to
    # two v_fma_f32 with it); only the host pass warns that it does not know it
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def needs_build() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and not needs_build():
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
