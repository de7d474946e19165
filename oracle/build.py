"""Build step of the CPU oracle: plain g++, -O2, no fast-math, no contraction."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "stmf_oracle.cpp")
OUT = os.path.join(_HERE, "liboracle.so")
FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-fno-fast-math", "-msse2", "-mfpmath=sse", "-fopenmp", "-Wall"]


def build(force: bool = True) -> str:
    if not force and os.path.exists(OUT) and os.path.getmtime(OUT) >= os.path.getmtime(SRC):
        return OUT
    tmp = OUT + ".tmp"
    subprocess.run(["g++", *FLAGS, SRC, "-o", tmp], check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
