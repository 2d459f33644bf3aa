"""Compile the generator library libgraphgen.so in place (host + gfx950)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libgraphgen.so")
SOURCES = [os.path.join(HERE, "csrc", "gg_host.cpp"), os.path.join(HERE, "csrc", "gg_device.hip")]


def build(verbose=False):
    cmd = [
        "hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        "-pthread", "-o", LIB + ".tmp",
    ] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
