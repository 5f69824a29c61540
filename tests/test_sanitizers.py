"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the C
oracle (small grids, every source kind, the switch-on, both pole rules), the
library's host setup (coefficient and source tables, tortoise inversion,
step rule), and the library's host entry points driven from C.  Compiled
with gcc / g++ here; no GPU."""
import os
import subprocess

import pytest

from paper_1206_0270_amd.csrc import build as libbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "_build")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd):
    return subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=300)


def test_oracle_under_sanitizers():
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "oracle_sanitized")
    subprocess.run(["gcc", "-std=c99", *SAN, "-ffp-contract=off", "-fcx-fortran-rules",
                    os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), "-o", exe, "-lm"], check=True)
    r = _run([exe])
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


@pytest.mark.parametrize("args", [
    ["1", "0.9", "-2", "2", "201", "17", "-20", "30", "1", "8.1"],
    ["1", "0.99", "-2", "8", "101", "33", "-300", "300", "2", "10"],
    ["1", "0.0", "1", "-2", "77", "16", "-20", "30", "3", "7"],
    ["1", "0.5", "0", "0", "60", "5", "-10", "40"],
])
def test_host_setup_under_sanitizers(args):
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "host_setup_sanitized")
    csrc = os.path.join(ROOT, "paper_1206_0270_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + csrc,
                    os.path.join(ROOT, "tests", "host_setup_check.cpp"), os.path.join(csrc, "tk_setup.cpp"),
                    "-o", exe], check=True)
    r = _run([exe] + args)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, \
        r.stderr[-2000:]


def test_host_library_entry_points_under_sanitizers():
    # the library's host code (C ABI, validation, work lists, layout, post-
    # processing) rebuilt with the sanitizers and driven from C without a
    # device; the kernels' objects are linked as built
    kobjs = [os.path.join(BUILD, k + ".o") for k in libbuild.HIP_SOURCES]
    if not all(os.path.exists(k) for k in kobjs):
        pytest.skip("build the library first (its kernels' objects are linked here)")
    out = os.path.join(BUILD, "san")
    os.makedirs(out, exist_ok=True)
    csrc = os.path.join(ROOT, "paper_1206_0270_amd", "csrc")
    inc = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")]
    objs = []
    for f in ("tk_api", "tk_setup", "tk_post"):
        o = os.path.join(out, f + ".o")
        subprocess.run(["g++", "-std=c++17", "-fPIC", *SAN, *inc, "-c", os.path.join(csrc, f + ".cpp"), "-o", o],
                       check=True)
        objs.append(o)
    lib = os.path.join(out, "libtk.so")
    subprocess.run(["g++", "-shared", "-fsanitize=address,undefined", *objs, *kobjs, "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib", "-o", lib], check=True)
    exe = os.path.join(out, "abi_driver")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", *SAN, *inc,
                    os.path.join(ROOT, "tests", "abi_sanitize_driver.c"), "-o", exe, "-L" + out, "-ltk",
                    "-Wl,-rpath," + out, "-lm"], check=True)
    r = _run([exe])
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr[-3000:]
