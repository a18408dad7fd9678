"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so, and the same
source with OpenMP into oracle/liboracle_omp.so.

The oracle is compiled with gcc, -O3, no fused multiply-add contraction and no fast-math,
so that every operation is evaluated in the order written.  The OpenMP build runs the
independent rows and lines of each loop on all host cores; every item is computed from
the same inputs by the same operations, so both builds give identical results.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ccref.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")
FLAGS = ["-O3", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def _build_one(out, extra, verbose):
    cmd = ["gcc"] + FLAGS + extra + ["-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose=False):
    _build_one(LIB, ["-Wno-unknown-pragmas"], verbose)
    _build_one(LIB_OMP, ["-fopenmp"], verbose)
    return LIB


def ensure_built(parallel=False):
    out = LIB_OMP if parallel else LIB
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
        build()
    return out


if __name__ == "__main__":
    print(build(verbose=True))
