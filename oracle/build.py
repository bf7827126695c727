"""Build the FP64 CPU oracle shared library (test infrastructure only).

``python oracle/build.py`` compiles ``moto_oracle.c`` with the system C
compiler into ``oracle/libmoto_oracle.so``.  Plain ``-O2``: the oracle is
meant to be obviously correct, not fast.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "moto_oracle.c")
LIB = os.path.join(HERE, "libmoto_oracle.so")


def build(verbose: bool = False) -> str:
    cc = os.environ.get("CC", "gcc")
    cmd = [cc, "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
