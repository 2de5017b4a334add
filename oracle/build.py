"""Build the CPU oracle (test infrastructure only) into oracle/libqoz_ref.so.

Plain g++, -O2, no FP contraction and no fast-math, so every FP32 operation
of the predictor and quantizer is rounded on its own, in source order.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["ref_core.cpp", "ref_huffman.cpp", "ref_stream.cpp",
           "ref_metrics.cpp", "ref_tune.cpp"]
LIB = os.path.join(HERE, "libqoz_ref.so")


def build(verbose=False):
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
