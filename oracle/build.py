"""Build the C oracle into oracle/liboracle.so with gcc, and the same sources
with OpenMP into oracle/liboracle_omp.so (the host-core timing of the
benchmark's CPU baseline: rows of a step on several threads, the same
per-site arithmetic).

Test infrastructure only.  Plain -O2 with -ffp-contract=off, so the oracle's
rounding follows the source expression by expression.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, "lbm_oracle.c"), os.path.join(HERE, "lbm_oracle_q9.c")]
    base = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared"]
    for lib, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        cmd = base + extra + ["-o", lib + ".tmp", *srcs, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
