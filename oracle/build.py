"""Build the oracle's C part (test infrastructure only).

Compiles ``oracle/jacobi.c`` with gcc into ``oracle/liboracle.so``.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark load it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jacobi.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
