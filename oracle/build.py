"""Build the C oracle into oracle/liboracle.so with gcc.

Test infrastructure only.  Plain -O2 with -ffp-contract=off, so the oracle's
rounding follows the source expression by expression.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, "lbm_oracle.c"), os.path.join(HERE, "lbm_oracle_q9.c")]
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared",
           "-o", LIB + ".tmp", *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
