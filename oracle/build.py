"""Build the FP64 CPU oracle (plain C, gcc -O2, no fast-math, no intrinsics).

Test infrastructure: the oracle library is loaded only by tests, the smoke
check and the benchmark's CPU-baseline leg.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bloch_oracle.c")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "liboracle.so")


def build(verbose: bool = False, src: str = SRC, out: str = LIB, extra_flags=()) -> str:
    """extra_flags: appended to the compile line (the sanitizer test's
    -fsanitize options); the arithmetic flags stay as they are."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-fno-fast-math",
           "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra", *extra_flags, "-o", tmp, src,
           "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
