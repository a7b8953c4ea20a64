"""Build the HIP library paper_2103_02119_amd/liblbm.so for gfx950.

Compiles the device kernels (csrc/lbm_tile.hip, lbm_tile2.hip, lbm_march.hip,
lbm_aux.hip, nn_kernels.hip) and the host side of the C ABI (csrc/lbm_api.hip
for include/lbm.h, csrc/lbm_batch.hip for include/lbm_batch.h) with hipcc,
one object per source in parallel, into one shared library that links only
against the HIP runtime.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = [os.path.join(CSRC, f) for f in
           ("lbm_tile.hip", "lbm_tile2.hip", "lbm_march.hip", "lbm_aux.hip", "lbm_api.hip",
            "lbm_batch.hip", "nn_kernels.hip")]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC",
         # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # fuse a*b+c only within one source expression, so every inlined copy
         # of the collision (fast / generic path, single / batch kernel, one or
         # two steps per launch, any launch shape) rounds identically
         "-ffp-contract=on",
         "-Wall", "-Wno-unused-function"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.basename(src).replace(".hip", ".o"))
        cmd = [cc, f"--offload-arch={ARCH}", *FLAGS, "-I", os.path.join(ROOT, "include"),
               *extra, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
