"""Build the FP64 CPU oracle (test infrastructure only) with gcc.

The oracle is a plain C99 library, ``liborc_rbsog.so``, built next to its
source.  Nothing in the HIP library links or loads it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rbsog_oracle.c")
LIB = os.path.join(HERE, "liborc_rbsog.so")


def build_oracle(verbose: bool = False) -> str:
    """Compile the oracle; returns the path of the shared library."""
    cmd = [
        "gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
        "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))
