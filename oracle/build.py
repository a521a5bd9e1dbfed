"""Build the CPU oracle library (test infrastructure only).

Compiles oracle/ckks_oracle.c with gcc into oracle/liboracle.so.  Only tests,
the smoke check and the CPU-baseline leg of the benchmark load the result.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckks_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-Wall", "-Wno-unused-function",
           SRC, "-o", tmp, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
