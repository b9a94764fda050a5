"""Build the plain C oracle (test infrastructure) into oracle/liboracle.so.

The flags matter for bit-exactness: no fused multiply-add (-ffp-contract=off),
IEEE semantics (-fno-fast-math), default round-to-nearest-even.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tmd_oracle.c")
SRCS = [SRC, os.path.join(HERE, "rans_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall", "-Wextra",
          "-shared", "-fPIC"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, *SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
