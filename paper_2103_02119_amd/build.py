"""Build the HIP library paper_2103_02119_amd/liblbm.so for gfx950.

Compiles csrc/lbm_kernels.hip (device kernels), csrc/lbm_api.hip (the C ABI
of include/lbm.h), csrc/lbm_batch.hip (the batch ABI of include/lbm_batch.h)
and csrc/nn_kernels.hip (the warm-start network, include/lbm_nn.h) with hipcc into one shared library that links only
against the HIP runtime.
"""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = [os.path.join(CSRC, "lbm_kernels.hip"), os.path.join(CSRC, "lbm_api.hip"),
           os.path.join(CSRC, "lbm_batch.hip"), os.path.join(CSRC, "nn_kernels.hip")]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # fuse a*b+c only within one source expression, so every inlined
           # copy of the collision (fast / generic path, single / batch kernel,
           # any launch shape) rounds identically
           "-ffp-contract=on",
           "-Wall", "-Wno-unused-function",
           "-I", os.path.join(ROOT, "include"), *extra, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
