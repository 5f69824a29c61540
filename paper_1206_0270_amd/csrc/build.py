"""Build libtk.so (the HIP library) in-tree for gfx950.

hipcc compiles the kernels (tk_kernels.hip, tk_layer.hip) and the host C++ (setup, C ABI)
and links them into paper_1206_0270_amd/libtk.so.  Objects go to _build/.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libtk.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_SOURCES = ["tk_kernels.hip", "tk_layer.hip"]
HOST_SOURCES = ["tk_setup.cpp", "tk_api.cpp", "tk_post.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter",
          "-I" + os.path.join(ROOT, "include")]
# device code: gfx950 only; packed FP32 instructions disabled.  Multiply-adds
# are fused per source expression (contract=on), never across statements:
# with cross-statement fusion the compiler fuses differently in different
# inlined copies of the same row update, and the result of a row would then
# depend on where the launch's tiling puts it.
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-ffp-contract=on", "-munsafe-fp-atomics"]


def run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False, extra=()):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        run([HIPCC, *COMMON, *DEVICE, *extra, "-c", os.path.join(HERE, src), "-o", obj], verbose)
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        run([HIPCC, *COMMON, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *extra, "-c",
             os.path.join(HERE, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = OUT + ".tmp"
    run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
