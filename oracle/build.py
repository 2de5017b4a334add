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
# the same sources with AddressSanitizer and UndefinedBehaviorSanitizer, for
# running the CPU tests under the sanitizers (host code only)
LIB_SAN = os.path.join(HERE, "libqoz_ref_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]


def build(verbose=False, sanitize=False):
    out = LIB_SAN if sanitize else LIB
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra"]
    if sanitize:
        cmd += SAN_FLAGS
    cmd += ["-o", out + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def sanitizer_runtime():
    """Path of the ASan runtime that must be preloaded into the Python
    process that loads LIB_SAN."""
    return subprocess.run(["g++", "-print-file-name=libasan.so"],
                          capture_output=True, text=True,
                          check=True).stdout.strip()


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
