"""Build the HIP library libdr.so for gfx950 in-tree (hipcc cross-compiles
without a GPU).  The translation units (the host side and small kernels in
dr_lib.hip, the L-templated kernels in dr_inst_*.hip, the host BVH builder)
compile in parallel into _build/ and link into one shared object."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdr.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ([os.path.join(CSRC, "dr_lib.hip")] + sorted(glob.glob(os.path.join(CSRC, "dr_inst_*.hip"))) +
           [os.path.join(CSRC, "dr_mixture.hip"), os.path.join(CSRC, "bvh_build.cpp")])
DEPS = SOURCES + [os.path.join(CSRC, h) for h in ("dr_device.h", "dr_adjoint.h", "dr_chain.h", "dr_machine.h",
                                                  "dr_kernels.h")] + [os.path.join(ROOT, "include", "dr.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
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


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-8000:]}")
    return obj


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and not needs_build():
        return LIB
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    # -z defs: a symbol left undefined (a launcher no unit instantiates) fails the link
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-z,defs", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
