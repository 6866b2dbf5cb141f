"""Build the test-only host library tests/host/_plan_host.so (g++, no GPU):
the library's host plan plus a CPU emulation of its device solve programs, and
C entry points over the step server's scheduling policy."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_plan_host.so")
SRCS = [os.path.join(HERE, "plan_emulate.cpp"), os.path.join(HERE, "serve_shim.cpp"),
        os.path.join(ROOT, "paper_2405_12484_amd", "csrc", "host_plan.cpp"),
        os.path.join(ROOT, "paper_2405_12484_amd", "csrc", "cms_plan.cpp")]
DEPS = SRCS + [os.path.join(ROOT, "paper_2405_12484_amd", "csrc", h) for h in ("plan.h", "serve_policy.h")]


def build():
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", *SRCS, "-o", OUT + ".tmp"]
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


def ensure():
    if not os.path.exists(OUT) or any(os.path.getmtime(s) > os.path.getmtime(OUT) for s in DEPS):
        build()
    return OUT


if __name__ == "__main__":
    build()
