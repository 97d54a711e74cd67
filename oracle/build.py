"""Build the CPU oracle's shared library (test infrastructure, plain C).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
the oracle; the product library never links or loads it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "greedy_oracle.c")
LIBRARY = os.path.join(HERE, "libgreedy_oracle.so")


def build(verbose: bool = False) -> str:
    """Compile greedy_oracle.c with gcc into libgreedy_oracle.so (always)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", LIBRARY + ".tmp", SOURCE]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIBRARY + ".tmp", LIBRARY)
    return LIBRARY


if __name__ == "__main__":
    print(build(verbose=True))
