"""Build step for the oracle: compiles spa_oracle.c into liboracle_spa.so.

Test infrastructure only (see spa_oracle.c).  Plain gcc, no fast-math, so the
libm tanh/atanh used are the IEEE-accurate ones.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spa_oracle.c")
LIB = os.path.join(HERE, "liboracle_spa.so")


def compile_oracle(src: str = SRC, out: str = LIB, extra=()) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Werror",
           *extra, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build() -> str:
    return compile_oracle()


if __name__ == "__main__":
    print(build())
