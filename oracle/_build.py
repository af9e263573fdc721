"""ORACLE - TEST INFRASTRUCTURE ONLY.  Compiles the plain-C FP64 SDF loop."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csdf.c")
LIB = os.path.join(HERE, "_csdf.so")


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-fno-fast-math", "-ffp-contract=off", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB
