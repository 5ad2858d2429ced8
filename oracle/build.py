"""Build the CPU oracle (plain C, gcc) into ``oracle/liboracle.so``.

Test infrastructure only: the library never links or loads this.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(src: str = SRC, out: str = LIB, extra_flags=()) -> str:
    """Compile ``src`` to the shared object ``out``; returns ``out``."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           *extra_flags, "-o", out, src]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(), file=sys.stderr)
