"""Build step for the CPU oracle library (test infrastructure only)."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ttie_oracle.cpp")
LIB = os.path.join(HERE, "libttie_oracle.so")

# -ffp-contract=off: no fused multiply-adds, so every FP64 operation rounds as written
FLAGS = ["-O2", "-ffp-contract=off", "-fopenmp", "-std=c++17", "-shared", "-fPIC", "-Wall"]


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        subprocess.run(["g++", *FLAGS, "-o", LIB, SRC], check=True)
    return LIB


if __name__ == "__main__":
    print(build())
