"""Build the oracle shared libraries (test infrastructure only).

Compiles oracle/*.cpp with g++ -O2 (IEEE semantics, no fast-math) and OpenMP
into oracle/_build/liboracle.so, and the same sources a second time with the
arithmetic type set to long double (x87 extended precision, 64-bit
significand) into oracle/_build/liboracle_ld.so: the extended-precision
reference that bounds the rounding of FP64 evaluations.  The second build
renames the internal namespace and binds its own symbols, so both libraries
can be loaded into one process.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")
LIB_LD = os.path.join(OUT_DIR, "liboracle_ld.so")
SOURCES = ["kinematics.cpp", "processes.cpp", "gluons.cpp", "quark_lines.cpp", "api.cpp"]
FLAGS = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unused-function"]


def _link(out, extra, verbose):
    cmd = FLAGS + extra + ["-o", out + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    _link(LIB, [], verbose)
    _link(LIB_LD, ["-DORC_REAL=long double", "-Dorc=orc_ld", "-Wl,-Bsymbolic"], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
