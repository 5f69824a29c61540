"""Build libtk.so (the HIP library) in-tree for gfx950.

hipcc compiles the kernels (tk_kernels.hip, tk_layer.hip) and the host C++ (setup, C ABI)
and links them into paper_1206_0270_amd/libtk.so.  Objects go to _build/.

Every kernel must run without spills: the build reads the compiler's resource
report of each kernel and fails if one uses scratch memory (register spills or
private arrays kept in memory) or accumulation registers (which, with no
matrix-core code here, only ever hold spilled values).  A spill inside a
divergent region saves and restores only the active lanes, and the cross-lane
column exchange reads a neighbour's register whatever that lane's state:
launch shapes that spilled are the only ones that ever computed wrong values
here.  A private array in scratch also turns register reads into memory
traffic inside the march.  The report goes to _build/kernel_resources.txt.
"""
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libtk.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_SOURCES = ["tk_kernels.hip", "tk_layer.hip", "tk_scratch.hip"]
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


_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]"
                     r"|VGPRs Spill|SGPRs Spill):\s*(\S+)")


def kernel_resources(text):
    """Per kernel (mangled name): VGPRs, AGPRs, scratch bytes per lane,
    occupancy and spill counts, from hipcc's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[key.split(" [")[0]] = int(val)
    return out


def compile_device(cmd, verbose):
    """Compile one HIP source with the resource report on; return the report."""
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    for line in p.stderr.splitlines():
        if "remark:" not in line and noise not in line and not line.strip().startswith(("|", "^")) \
                and not re.match(r"^\s*\d+\s*\|", line):
            print(line, file=sys.stderr)
    if p.returncode != 0:
        raise subprocess.CalledProcessError(p.returncode, cmd)
    return kernel_resources(p.stderr)


def build(verbose=False, extra=()):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    report = {}
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        report.update(compile_device([HIPCC, *COMMON, *DEVICE, *extra, "-Rpass-analysis=kernel-resource-usage", "-c",
                                      os.path.join(HERE, src), "-o", obj], verbose))
        objs.append(obj)
    with open(os.path.join(BUILD, "kernel_resources.txt"), "w") as f:
        for name, r in sorted(report.items()):
            f.write(f"{name} {r}\n")
    if not report:
        raise RuntimeError("no kernel resource report from hipcc")
    # No kernel here uses the matrix cores, so accumulation registers would
    # only hold spilled values, which are refused like scratch spills.
    bad = {k: v for k, v in report.items()
           if v.get("ScratchSize", 0) > 0 or v.get("VGPRs Spill", 0) > 0 or v.get("AGPRs", 0) > 0}
    if bad:
        raise RuntimeError("kernels spilling registers (to scratch memory or to accumulation registers) or keeping "
                           "private arrays in memory: " + "; ".join(f"{k}: {v}" for k, v in bad.items()))
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
