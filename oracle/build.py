"""Build the C oracle library (``liboracle.so``) with gcc.  Test infrastructure only."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vor_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
FILTER_SRC = os.path.join(HERE, "filter_exact.c")
FILTER_LIB = os.path.join(HERE, "libfilterexact.so")


def _gcc(src: str, lib: str, verbose: bool, extra=()) -> None:
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
           "-o", lib + ".tmp", src] + list(extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)


def build(verbose: bool = False) -> str:
    _gcc(SRC, LIB, verbose)
    _gcc(FILTER_SRC, FILTER_LIB, verbose, ["-fopenmp", "-lm"])
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
