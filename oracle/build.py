"""Build the CPU oracle library (plain C, gcc).  Test infrastructure only."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tm_oracle.c")
LIB = os.path.join(HERE, "libtm_oracle.so")


def build(verbose: bool = False) -> str:
    """Compile oracle/tm_oracle.c into oracle/libtm_oracle.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-fopenmp", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    """The library is missing or older than its source."""
    return not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)


if __name__ == "__main__":
    print(build(verbose=True))
