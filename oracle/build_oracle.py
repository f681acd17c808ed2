"""Compile the CPU oracle into oracle/liboracle.so with gcc.

Test infrastructure: the oracle is built here (and by ``__graft_entry__.build``)
so that tests and the benchmark's CPU-baseline leg can load it.  The flags keep
every floating-point operation a separately rounded IEEE-754 operation:
``-ffp-contract=off`` stops gcc from fusing a*b + c (its default is to fuse when
the target has FMA), ``-fno-fast-math`` keeps IEEE semantics.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "julia_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
