"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

The shipped build targets x86-64-v3 (AVX2), so the library built in one
container also loads on another host's CPU.  The CPU-baseline timing builds a
second copy for the CPU it runs on (-march=native) in a temporary directory.
Contraction stays off in both: Hamiltonian elements are compared bit for bit.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, native: bool = False, out: str = OUT) -> str:
    arch = "-march=native" if native else "-march=x86-64-v3"
    cmd = ["g++", "-O3", arch, "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", SRC, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
