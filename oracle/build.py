"""Build the CPU oracle shared library (oracle/liblbmref.so) with gcc.

TEST INFRASTRUCTURE ONLY: the oracle is what the HIP path is checked against.
It is compiled with FMA contraction off and no fast-math, so every rounding
step is the one written in lbmref.c.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbmref.c")
LIB = os.path.join(HERE, "liblbmref.so")

FLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
         "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle; with force=False, only when the library is missing or stale."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "lbmref.h"))):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", *FLAGS, "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
