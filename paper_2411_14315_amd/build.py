"""Build libhb.so (HIP kernels + C interface) for gfx950 in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhb.so")
SOURCES = ["hb_kernels.hip", "hb_host.cpp", "hb_mlp.hip", "hb_precond.hip", "hb_pod.hip"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = True) -> str:
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-result"]
    for src in SOURCES:
        obj = os.path.join(CSRC, src.rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [hipcc()] + common + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


SAN_DIR = os.path.join(HERE, "_san")
SAN_LIB = os.path.join(SAN_DIR, "libhb_san.so")


def asan_runtime() -> str:
    """Path of the compiler's AddressSanitizer runtime (for LD_PRELOAD)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    out = subprocess.run([os.path.join(rocm, "llvm", "bin", "clang"),
                          "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True, check=True)
    return out.stdout.strip()


def build_sanitized(verbose: bool = True) -> str:
    """The same library with AddressSanitizer and UndefinedBehaviorSanitizer
    in its host code only (the device code is built as usual), -O1, for
    running the host-side entry points (argument and mesh checks, the
    eigensolver) under the sanitizers on a machine without a GPU."""
    os.makedirs(SAN_DIR, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
              "-I", CSRC] + san
    objs = []
    for src in SOURCES:
        obj = os.path.join(SAN_DIR, src.rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [hipcc()] + common + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = SAN_LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950"] + san + \
          ["-shared-libsan", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        build_sanitized(verbose="-q" not in sys.argv)
    else:
        build(verbose="-q" not in sys.argv)
