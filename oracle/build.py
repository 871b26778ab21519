"""Compile the C oracle (test infrastructure) into ``oracle/libspegg_oracle.so``."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spegg_oracle.c")
LIB = os.path.join(HERE, "libspegg_oracle.so")


def build(verbose: bool = False) -> str:
    # -ffp-contract=off: probabilities must be the IEEE result of each
    # basic operation, with no fused multiply-add.
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-ffp-contract=off", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
