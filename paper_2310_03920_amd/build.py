"""Build libheffx.so (gfx950) in-tree with hipcc."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libheffx.so")
BUILD = os.path.join(HERE, "_build")
PEAK = os.path.join(HERE, "mfma_peak")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             # keep packed-FP32 instructions out of generated code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # MFMA accumulators in ordinary VGPRs: no AGPR <-> VGPR copies around
             # the K-stage loop of the block GEMM
             "-mllvm", "-amdgpu-mfma-vgpr-form"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_library(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    plan_o = os.path.join(BUILD, "heffx_plan.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-I", INCLUDE, "-I", CSRC, "-c",
          os.path.join(CSRC, "heffx_plan.cpp"), "-o", plan_o])
    objs.append(plan_o)
    kern_o = os.path.join(BUILD, "heffx_kernels.o")
    _run([hipcc] + HIP_FLAGS + ["-I", INCLUDE, "-I", CSRC, "-c",
                                os.path.join(CSRC, "heffx_kernels.hip"), "-o", kern_o])
    objs.append(kern_o)
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    # matrix-core throughput microbenchmark (roofline denominators measured on the GPU)
    _run([hipcc] + [f for f in HIP_FLAGS if f != "-fPIC"] + ["-o", PEAK, os.path.join(CSRC, "mfma_peak.hip")])
    return LIB


if __name__ == "__main__":
    build_library()
    sys.exit(0)
