"""Build the CPU oracle library (test infrastructure only).

    python oracle/build.py

compiles ``hoszp_ref.c`` with gcc into ``oracle/libhoszp_ref.so``.  Strict
IEEE binary64 evaluation: no FMA contraction, no fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hoszp_ref.c")
LIB = os.path.join(HERE, "libhoszp_ref.so")

CFLAGS = ["-std=gnu11", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wextra", "-Werror"]


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
