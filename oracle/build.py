"""Compile the C part of the oracle (test infrastructure only).

``python -m oracle.build`` or ``oracle.build.build()`` writes
``oracle/_lbm_oracle.so`` with gcc, OpenMP and IEEE double arithmetic
(no fast-math, no FMA contraction).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
OUT = os.path.join(HERE, "_lbm_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-std=c11",
           "-Wall", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


def ensure_built() -> str:
    if not os.path.exists(OUT) or os.path.getmtime(OUT) < os.path.getmtime(SRC):
        build()
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
