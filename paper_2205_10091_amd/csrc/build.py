"""Build libtcx.so (host C++ and HIP kernels for gfx950) in-tree.

    python paper_2205_10091_amd/csrc/build.py

Every HIP translation unit is compiled with the packed-FP32 target feature
disabled.  Host-only sources are compiled by hipcc as plain C++.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libtcx.so")
BUILD = os.path.join(ROOT, "_build")

HOST = ["network.cpp", "path.cpp", "plan.cpp", "slice.cpp", "capi_host.cpp"]
DEVICE = ["exec.hip", "serve.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", os.path.join(ROOT, "include"),
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
DEVFLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops", "-ffp-contract=fast"]


def run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HOST:
        obj = os.path.join(BUILD, src + ".o")
        run([HIPCC, "-c", *COMMON, os.path.join(HERE, src), "-o", obj])
        objs.append(obj)
    for src in DEVICE:
        obj = os.path.join(BUILD, src + ".o")
        run([HIPCC, "-c", "-x", "hip", *COMMON, *DEVFLAGS, os.path.join(HERE, src), "-o", obj])
        objs.append(obj)
    tmp = OUT + ".tmp"
    run([HIPCC, "-shared", "--offload-arch=gfx950", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    sys.exit(0 if build() else 1)
