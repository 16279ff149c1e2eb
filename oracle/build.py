"""Compile the C oracle into oracle/libpst_oracle.so (host compiler only).

Generic x86-64 code (no -march=native): the library is built here and may run
on another host.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pst_oracle.c")
LIB_PATH = os.path.join(HERE, "libpst_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", LIB_PATH + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
