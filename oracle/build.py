"""Compile the plain C oracle into oracle/liboracle.so (gcc, host only).

The oracle is test infrastructure: only the test suite, the smoke check and
the CPU-baseline leg of the benchmark load it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "oracle.c")]


def build(force: bool = True) -> str:
    """Build liboracle.so; with force=False an existing library is kept."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-pthread", "-o", tmp] + SOURCES
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--keep" not in sys.argv))
