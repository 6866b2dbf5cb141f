"""Build libvhpd.so in-tree for gfx950.

Host prefactor code is plain C++ (g++ with OpenMP); kernels and the C ABI are
HIP, compiled by hipcc for gfx950 only.  Packed FP32 instructions are disabled
for device code (they are known to misbehave on this hardware generation in
some forms; hipcc's host pass warns that it ignores the feature).  Code object
version 5 keeps the kernels loadable by the HIP runtime that PyTorch ships,
which is the runtime the library shares with it in one process.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libvhpd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall", "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]
CXX_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-fopenmp", "-Wall", "-Wextra", "-march=x86-64-v2"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    o = os.path.join(BUILD, "host_plan.o")
    _run(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "host_plan.cpp"), "-o", o])
    objs.append(o)
    o = os.path.join(BUILD, "cms_plan.o")
    _run(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "cms_plan.cpp"), "-o", o])
    objs.append(o)
    for src in ("kernels.hip", "api.hip", "serve.hip", "adjoint.hip", "embed.hip", "noalloc.hip", "gn.hip",
                "iface_factor.hip"):
        o = os.path.join(BUILD, src.replace(".hip", ".o"))
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-mcode-object-version=5", "-shared", "-fPIC", "-o", tmp, *objs, "-lgomp",
          f"-L{ROCM_LIB}", "-lrocsolver", "-lrocblas", f"-Wl,-rpath,{ROCM_LIB}"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
