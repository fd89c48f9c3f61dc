"""Builds libpcoll.so for gfx950 in this directory.

Device translation units (*.hip) are compiled by hipcc for gfx950 only, in
parallel; the host runtime (*.cpp) by g++ against the HIP runtime headers;
hipcc links the shared library.  Flags that matter for the numerics:
  -ffp-contract=off   no fused multiply-add: every add / multiply rounds
                      once, as the accumulation order requires;
  no fast-math        correctly rounded binary32 division, denormals kept;
and, for the hardware: packed FP32 instructions are disabled, and the
atomic optimizer is off so that the prefetched tile claim stays
asynchronous.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libpcoll.so")
OBJ = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIP_SOURCES = ["reduce_f32.hip", "reduce_i32.hip", "reduce_bf16.hip",
               "reduce_e4m3.hip", "reduce_e5m2.hip", "reduce_mx.hip",
               "aux.hip", "noalloc.hip"]
CPP_SOURCES = ["runtime.cpp", "tuning.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-function",
]
CXX_FLAGS = [
    "-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra",
    "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" +
                           r.stdout + r.stderr)
    return r


def build(verbose=False, jobs=None):
    """Compiles every source and links libpcoll.so; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    inc = ["-I" + CSRC, "-I" + INCLUDE]
    cmds = []
    objs = []
    for src in HIP_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        cmds.append([hipcc, *HIPCC_FLAGS, *inc, "-c",
                     os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for src in CPP_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        cmds.append(["g++", *CXX_FLAGS, *inc, "-c", os.path.join(CSRC, src),
                     "-o", o])
        objs.append(o)
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, _ in zip(cmds, ex.map(_run, cmds)):
            if verbose:
                print(" ".join(cmd), flush=True)
    tmp = LIB + ".tmp"
    link = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs,
            "-o", tmp, "-ldl"]
    _run(link)
    if verbose:
        print(" ".join(link), flush=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
