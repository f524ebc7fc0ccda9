"""Build libtnq.so (host C++ + gfx950 HIP kernels) in-tree with hipcc."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtnq.so")
SOURCES = ["network.cpp", "planner.cpp", "passes.cpp", "program.cpp", "fixedpoint.cpp", "slicing.cpp", "kernels.hip", "runtime.hip"]
ARCH = os.environ.get("TNQ_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC, "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          # keep the compiler from emitting packed FP32 arithmetic
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# Host sanitizer variant (AddressSanitizer + UndefinedBehaviorSanitizer on the
# host code only; the GPU code is built as usual): libtnq_san.so, for running
# the CPU test suite under the sanitizers (LD_PRELOAD the clang ASan runtime and
# point TNQ_LIB at this library).
SAN_BUILD = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(HERE, "libtnq_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def _compile(src: str, verbose: bool, sanitize: bool = False) -> str:
    obj = os.path.join(SAN_BUILD if sanitize else BUILD, src + ".o")
    cmd = ["hipcc", "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON
    if sanitize:
        cmd = [c for c in cmd if c != "-O3"] + ["-O1"] + SAN_FLAGS
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    os.makedirs(SAN_BUILD if sanitize else BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, sanitize), SOURCES))
    out = SAN_LIB if sanitize else LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libasan"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
