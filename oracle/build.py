"""Build the C oracle (test infrastructure) with the host C compiler."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ref.c")
LIB_PATH = os.path.join(HERE, "libref.so")


def build_oracle(openmp: bool = True) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off"]
    if openmp:
        cmd.append("-fopenmp")
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd += [SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build_oracle())
