"""Build step for the CPU oracle: oracle/*.c -> liboracle.so (gcc, -O2, OpenMP).

Test infrastructure only; called by __graft_entry__.build() and, when the
library is missing, by the oracle's own loader.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, f) for f in ("ils_oracle.c", "mlp_oracle.c", "sparse_oracle.c")]
SRC = SRCS[0]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", *SRCS, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
