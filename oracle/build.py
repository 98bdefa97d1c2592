"""Compile the oracle's C part (test infrastructure; gcc + OpenMP)."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    src = os.path.join(_HERE, "csrc", "efm_direct.c")
    out = os.path.join(_HERE, "_efm_direct.so")
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, src])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
