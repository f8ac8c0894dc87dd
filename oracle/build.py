"""Build the plain-C oracle (test infrastructure) into oracle/libugks_oracle.so
and its dual-number tangent build into oracle/libugks_oracle_tl.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ugks_oracle.c")
SRC_TL = os.path.join(HERE, "ugks_oracle_tl.cpp")
LIB = os.path.join(HERE, "libugks_oracle.so")
LIB_TL = os.path.join(HERE, "libugks_oracle_tl.so")
FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall",
         "-Wno-unused-function"]


def build(verbose=False):
    for cmd, out in ((["gcc", "-std=c99"] + FLAGS + ["-o", LIB + ".tmp", SRC, "-lm"], LIB),
                     (["g++", "-std=c++17"] + FLAGS + ["-o", LIB_TL + ".tmp", SRC_TL, "-lm"], LIB_TL)):
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
