"""Builds the seeded input generator (libfx.so) with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose=False):
    out = os.path.join(HERE, "libfx.so")
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", out + ".tmp", os.path.join(HERE, "fx.c"), "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
