"""Build the FP64 CPU oracle (test infrastructure) into oracle/liblgt_oracle.so.

Plain C99 + OpenMP, built with gcc; no HIP headers, no source shared with the
library.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liblgt_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "lgt_oracle.c")
    tmp = SO + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
