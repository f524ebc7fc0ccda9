"""Compile the FP64 oracle (plain C + OpenMP) into oracle/liboracle.so.

Test infrastructure: the oracle checks the product, it is never part of it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


# Sanitizer variant: AddressSanitizer + UndefinedBehaviorSanitizer, built with
# ROCm's clang so that it shares one ASan runtime with the sanitized libtnq
# (selected with ORACLE_LIB).
SAN_LIB = os.path.join(HERE, "liboracle_san.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = SAN_LIB if sanitize else LIB
    tmp = out + ".tmp%d" % os.getpid()
    if sanitize:
        cmd = [CLANG, "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE", "-Wall", "-Wextra",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
               "-shared-libasan", "-o", tmp, SRC, "-lm"]
    else:
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
               "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
