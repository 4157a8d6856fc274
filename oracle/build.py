"""Build the FP64 CPU oracle (test infrastructure only) with gcc.

The oracle is compiled with -O2 -ffp-contract=off so that every floating-point
operation is rounded as written in su3ref.c, and with OpenMP so that the
independent links of one checkerboard pass can be updated on all host cores.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsu3ref.so")


def build(force: bool = True) -> str:
    src = os.path.join(HERE, "su3ref.c")
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(src):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-pipe", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
