"""Build the FP64 CPU oracle (test infrastructure only) with gcc.

The oracle is plain C99 compiled at -O2 without fast-math, so its
arithmetic follows IEEE double precision in source order (liboracle.so,
used for every parity check).  The same source compiled with -fopenmp
(liboracle_omp.so) spreads the pair enumeration and pair sums over threads;
it serves only the benchmark's CPU-baseline timing.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "h4d_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def _gcc(out: str, extra, verbose: bool) -> str:
    cmd = ["gcc", "-std=gnu11", "-O2", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter"] + extra + ["-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


def build(verbose: bool = False) -> str:
    """The parity build, and beside it the OpenMP timing build."""
    _gcc(LIB_OMP, ["-fopenmp"], verbose)
    return _gcc(LIB, [], verbose)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
