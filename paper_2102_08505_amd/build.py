"""Build libellsp2.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libellsp2.so")
SOURCES = ["ell_api.hip", "ell_kernels.hip", "ell_band.hip", "ell_band16.hip", "ell_sym16.hip", "dense.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # every multiply-add is the fma() or the separate operations written in the source
    "-ffp-contract=off",
    "-fno-gpu-flush-denormals-to-zero",
    "-fno-fast-math",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]

# The matrix-core kernels keep their accumulators in VGPRs: with the
# compiler's AGPR choice they are copied between the two files every step (the
# dense GEMMs: all 128 accumulator registers twice per k-slice, and the FP64
# GEMM then needs 344 registers, one wavefront per SIMD, against 222).
EXTRA_FLAGS = {"ell_band16.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
               "ell_sym16.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
               "dense.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def build(verbose=False, jobs=4):
    hipcc = os.environ.get("HIPCC", "hipcc")
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src.replace(".hip", ".o"))
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [hipcc, *HIPCC_FLAGS, *EXTRA_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, cwd=CSRC, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    failed = []
    for p, src in procs:
        _, err = p.communicate()
        if p.returncode != 0:
            failed.append((src, err))
        elif verbose and err.strip():
            print(err, file=sys.stderr)
    if failed:
        for src, err in failed:
            print(f"--- {src}\n{err}", file=sys.stderr)
        raise RuntimeError("hipcc failed: " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
