"""Build libatrapos.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libatrapos.so")
SOURCES = ["kernels.hip", "engine.cpp", "planner.cpp", "otree.cpp", "serve.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread",
    "--offload-arch=gfx950",
    # packed FP32 instructions stay off in every device pass
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


# host code instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
# (device code is not: GPU sanitizers are not used); load it with the clang
# ASan runtime preloaded, see sanitizer_env()
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-g"]
LLVM = os.environ.get("ATP_LLVM", "/opt/rocm/llvm")


def asan_runtime() -> str:
    """The clang ASan runtime that a sanitizer build expects to be preloaded."""
    import glob
    libs = sorted(glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not libs:
        raise RuntimeError("clang ASan runtime not found under " + LLVM)
    return libs[-1]


def build(verbose: bool = False, sanitize: bool = False, out: str | None = None) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    lib = out or (os.path.join(HERE, "_san", "libatrapos.so") if sanitize else LIB)
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if sanitize else []), "-x", "hip", *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose and r.stderr.strip():
        # the host pass does not know the packed-fp32 feature; that warning is expected
        lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    san = "--sanitize" in sys.argv[1:]
    print(build(verbose=True, sanitize=san))
    if san:
        print("load with LD_PRELOAD=" + asan_runtime() + " ATP_LIBRARY=<the path above>")
