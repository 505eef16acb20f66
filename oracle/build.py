"""Build the oracle shared library (plain C, gcc).  Test infrastructure."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpivco_ref.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, f) for f in ("pivco_ref.c", "golomb_ref.c", "fse_ref.c")]
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-Werror", "-fPIC", "-shared",
           *srcs, "-lm", "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
