"""Build step for the oracle: compiles spa_oracle.c (flooding), layered_oracle.c
(layered schedule) and minsum_oracle.c (min-sum rule, both schedules) into
liboracle_spa.so, and spa_oracle.c once more with its check node evaluated in
80-bit long double (ORACLE_CHECK_LD) into liboracle_spa_ld.so.

Test infrastructure only (see spa_oracle.c).  Plain gcc, no fast-math, so the
libm tanh/atanh used are the IEEE-accurate ones.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spa_oracle.c")
SRC_LAYERED = os.path.join(HERE, "layered_oracle.c")
SRC_MINSUM = os.path.join(HERE, "minsum_oracle.c")
LIB = os.path.join(HERE, "liboracle_spa.so")
LIB_LD = os.path.join(HERE, "liboracle_spa_ld.so")


def compile_oracle(src=(SRC, SRC_LAYERED, SRC_MINSUM), out: str = LIB, extra=()) -> str:
    """Compile one source file (a path) or several (a sequence) into `out`."""
    srcs = [src] if isinstance(src, str) else list(src)
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Werror",
           *extra, *srcs, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def compile_long_double(out: str = LIB_LD) -> str:
    return compile_oracle(SRC, out, extra=("-DORACLE_CHECK_LD",))


def build() -> str:
    compile_long_double()
    return compile_oracle()


if __name__ == "__main__":
    print(build())
