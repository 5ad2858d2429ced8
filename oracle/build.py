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


def build_native(out: str, src: str = SRC) -> str:
    """The same source compiled as the paper compiled its sorters for timing
    (gcc -O3 -march=native, Section 4.1), for the host that runs it.  Used
    only to time the oracle as a CPU baseline; correctness tests load LIB."""
    cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-shared", "-fPIC", "-o", out, src]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(), file=sys.stderr)
