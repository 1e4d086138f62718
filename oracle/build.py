"""Compile the C oracle (test infrastructure) with gcc."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build():
    src = os.path.join(_HERE, "oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
