"""Build the oracle's C simulator (test infrastructure only).

    python oracle/build.py

Writes ``oracle/_qwo.so`` with gcc (OpenMP over amplitude loops).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qwo.c")
OUT = os.path.join(HERE, "_qwo.so")


OUT_ASAN = os.path.join(HERE, "_qwo_asan.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """``sanitize``: ``_qwo_asan.so`` with AddressSanitizer and
    UndefinedBehaviorSanitizer (load it with QWO_LIB and LD_PRELOAD of gcc's
    libasan.so; see the package build module)."""
    out = OUT_ASAN if sanitize else OUT
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer"] if sanitize else []
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", *san,
           "-fno-fast-math", "-ffp-contract=off", "-fcx-limited-range", SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
