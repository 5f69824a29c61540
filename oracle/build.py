"""Build the oracle shared libraries (plain C, gcc).

TEST INFRASTRUCTURE: the oracle is only loaded by tests/, by the smoke check
and by the CPU-baseline leg of bench.py.

Two builds of the one source file:
  liboracle_f64.so  REAL = double       (the parity reference)
  liboracle_ld.so   REAL = long double  (80-bit x87, for rounding checks)
Both use -ffp-contract=off (no fused multiply-add contraction) and
-fcx-fortran-rules (plain complex products, no C99 Annex G recovery calls).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "teuk_oracle.c")
LIBS = {
    "f64": os.path.join(HERE, "liboracle_f64.so"),
    "ld": os.path.join(HERE, "liboracle_ld.so"),
}


BASE_FLAGS = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp",
              "-ffp-contract=off", "-fcx-fortran-rules", "-Wall", "-Wextra",
              "-Wno-unused-parameter"]


def build_one(src, out, long_double=False):
    """Compile one build of the oracle source (also used by tests that
    compile deliberately altered copies)."""
    cmd = list(BASE_FLAGS) + (["-DOR_LONG_DOUBLE"] if long_double else [])
    subprocess.run(cmd + [src, "-o", out, "-lm"], check=True)


def build(verbose=False):
    base = list(BASE_FLAGS)
    for kind, out in LIBS.items():
        cmd = list(base)
        if kind == "ld":
            cmd.append("-DOR_LONG_DOUBLE")
        tmp = out + ".tmp"
        cmd += [SRC, "-o", tmp, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
