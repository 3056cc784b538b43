"""Build the gfx950 shared library ``liblgf.so`` in-tree with hipcc.

``python -m paper_1305_3440_amd.build`` (or ``build()``) always recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_PATH = os.path.join(PKG, "liblgf.so")

SOURCES = ["lgf_kernels.hip", "lgf_fixed.hip", "lgf_ensemble_kernels.hip", "lgf_util.hip", "lgf_anneal.hip",
           "lgf_api.cpp", "lgf_ensemble_api.cpp"]

ARCH = "gfx950"

# -packed-fp32-ops: keep the compiler from forming packed FP32 instructions
# (v_pk_*_f32); ordinary scalar FP32 code is generated instead.
# -ffp-contract=on: multiply-adds are fused only within one source expression,
# decided before inlining, so a helper (the site update, reunitarization, the
# theta of a site) gives the same bits in every kernel it is inlined into -- the
# sweep, its fused-measurement variant, the measurement and the ensemble
# kernels agree bit for bit.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the gfx950 library cannot be built")
    return exe


def build(verbose: bool = False, extra_flags=()) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmds.append([hipcc, "-x", "hip", *HIP_FLAGS, *extra_flags, "-I", INCLUDE, "-I", CSRC, "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)

    def compile_one(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    # the translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as pool:
        for f in [pool.submit(compile_one, c) for c in cmds]:
            f.result()
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
