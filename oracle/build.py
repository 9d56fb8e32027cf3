"""Build the CPU oracle shared library (test infrastructure only).

gcc -O2 -ffp-contract=off: no fused multiply-add and no fast-math, so the
oracle's rounding is plain IEEE round-to-nearest per operation.  -fopenmp
lets the timing baseline spread the loops over atoms across host threads
(ora_set_threads; one thread by default).

build_sanitized() builds the same source with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; the oracle has no GPU code) into
a separate file; setting ORACLE_LIB to a library's path makes the ctypes
binding load that library instead of liboracle.so (the test that runs the
oracle's pins under the sanitizers does this, with the ASan runtime
preloaded into the interpreter).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
FLAGS = ["-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall", "-Wextra", "-fPIC",
         "-shared", "-fopenmp"]
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", *FLAGS, "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_sanitized(out: str, verbose: bool = False) -> str:
    """The oracle with ASan + UBSan (same rounding flags, -O1) at `out`."""
    cmd = ["gcc", "-O1", *FLAGS, *SANITIZE, "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


def ensure_built() -> str:
    override = os.environ.get("ORACLE_LIB")
    if override:
        return override
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
