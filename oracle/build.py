"""Build the CPU oracle (test infrastructure) as ``oracle/liboracle.so`` with g++.

IEEE float32 semantics are required: no FMA contraction, no fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tsdf_oracle.cpp")
OUT = os.path.join(HERE, "liboracle.so")
FLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fno-finite-math-only",
         "-fPIC", "-shared", "-Wall", "-Wextra"]


# The sanitized build (AddressSanitizer + UndefinedBehaviorSanitizer) uses
# ROCm's clang++, whose sanitizer runtime is the one the sanitized libtsdf.so
# expects: one process cannot hold two different ASan runtimes.
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SANITIZED_OUT = os.path.join(HERE, "liboracle_sanitized.so")
SANITIZE_FLAGS = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = SANITIZED_OUT if sanitize else OUT
    cmd = ([CLANGXX, *FLAGS, *SANITIZE_FLAGS] if sanitize else ["g++", *FLAGS]) + \
        [SRC, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
