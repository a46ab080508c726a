"""Compile the FP64 CPU oracle (``mdlj_oracle.c``) into ``liboracle.so``.

Test infrastructure only: the test-suite, the smoke check and the CPU
baseline of the benchmark load this library; the HIP library never does.
Built with ``-ffp-contract=off`` so every multiply and add rounds on its
own, as the definitions in ``mdlj_oracle.c`` are written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mdlj_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-Wno-unused-parameter", SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
