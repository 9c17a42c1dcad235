"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so.

Compiles oracle/so3_oracle.c twice with gcc (double and x87 long double) and
links both into one shared library.  No -ffast-math and no -march=native: the
library must give IEEE results and run on any x86-64 host.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "so3_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    """Compile the oracle; returns the path of the shared library."""
    objs = []
    for tag, defs in (("f64", []), ("f80", ["-DSO3O_LONG_DOUBLE"])):
        obj = os.path.join(HERE, f"so3_oracle_{tag}.o")
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-fopenmp", "-fvisibility=hidden",
               "-Wall", "-Wno-unused-function", *defs, "-c", SRC, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-shared", "-fopenmp", "-o", tmp, *objs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
