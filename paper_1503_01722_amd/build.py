"""Build the HIP library ``_lib/libomc.so`` for gfx950 with hipcc (in-tree).

Translation units:
  kernels_f32.hip  production transport (FP32, FP64 tally), fold, queue reset,
                   Philox debug kernel
  kernels_f64.hip  the parity instantiation, without FMA contraction
  runtime.cpp      host runtime and the C ABI of include/omc.h
  tables.cpp       closed-form physics tables (host, FP64)
  phantom_kernels.hip  voxel records and the CT mapping, without FMA contraction
  dn_kernels.hip   denoiser kernels (BF16 matrix-core convolutions, loss, Adam)
  dn_runtime.cpp   denoiser network, training and the C ABI of include/omc_dn.h
and, apart, ``_lib/libomc_ceilings.so`` from ceilings.hip: the microbenchmarks
of the ALU, HBM and FP64-atomic ceilings the measurement reports against.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libomc.so")
ARCH = os.environ.get("OMC_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
UNITS = {
    "kernels_f32.hip": ["-munsafe-fp-atomics"],
    "kernels_f64.hip": ["-munsafe-fp-atomics", "-ffp-contract=off"],
    "runtime.cpp": ["-ffp-contract=off"],
    "tables.cpp": ["-ffp-contract=off"],
    "phantom_kernels.hip": ["-ffp-contract=off"],
    "dn_kernels.hip": ["-munsafe-fp-atomics"],
    "dn_runtime.cpp": [],
}


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, extra):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc()] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd="/tmp")
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


# the ceiling microbenchmarks: a library of their own (measurement only)
CEIL_UNITS = {"ceilings.hip": []}
CEIL_LIB = os.path.join(LIBDIR, "libomc_ceilings.so")


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(UNITS) + len(CEIL_UNITS)) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), UNITS.items()))
        ceil_objs = list(ex.map(lambda kv: _compile(*kv), CEIL_UNITS.items()))
    tmp = CEIL_LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + ceil_objs
    r = subprocess.run(cmd, capture_output=True, text=True, cwd="/tmp")
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, CEIL_LIB)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True, cwd="/tmp")
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
