"""Compile the CPU oracle (plain C, gcc) into oracle/liboracle.so.

The oracle is test infrastructure: it is built so that the tests, the smoke
check and the CPU-baseline leg of the benchmark can load it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["ckks_oracle.c"]


def build(verbose=False):
    out = os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", tmp] + [os.path.join(HERE, s) for s in SOURCES] + ["-lquadmath", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
