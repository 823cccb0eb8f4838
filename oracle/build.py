"""Build the CPU oracle's shared library (test infrastructure only).

The oracle is compiled with gcc, never with hipcc, and links nothing from the
GPU library.  ``-ffp-contract=off`` keeps every multiply and add of the plain
substitution and of the Cholesky factorisation separately rounded, as the
sources' headers state.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "trsm_oracle.c")
CHOL_SRC = os.path.join(HERE, "chol_oracle.c")
SOURCES = (SRC, CHOL_SRC)
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle's C sources into ``liboracle.so`` next to them."""
    if (not force and os.path.exists(LIB)
            and all(os.path.getmtime(LIB) >= os.path.getmtime(s) for s in SOURCES)):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-pthread", *SOURCES, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv))
