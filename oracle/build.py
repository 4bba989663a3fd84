"""Compile the C oracle into oracle/liblrauv_oracle.so with gcc (no GPU code)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "lrauv_oracle.c"), os.path.join(HERE, "learned_oracle.c")]
LIB = os.path.join(HERE, "liblrauv_oracle.so")


def build(verbose: bool = False) -> str:
    srcs = [s for s in SRC if os.path.exists(s)]
    # -ffp-contract=off: no fused multiply-adds (the binary32 decisions of the
    # pairwise spawn must round every product)
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-fopenmp", "-Wall",
           "-Wextra",
           "-Wno-unused-parameter", *srcs, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
