"""Build libpkm.so (HIP for gfx950) in-tree: paper_1704_02357_amd/libpkm.so.

Every source is compiled with hipcc for gfx950 only, with packed-FP32 instructions
disabled, then linked into one shared library whose exports are declared in include/pkm.h.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpkm.so")

SOURCES = ["kernels_paint.hip", "kernels_fft.hip", "plan.hip", "runtime.hip", "host_math.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
          "-I" + os.path.join(ROOT, "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile_cmd(src: str) -> list[str]:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        return [HIPCC] + DEVICE + COMMON + ["-c", path, "-o", obj]
    return ["g++"] + COMMON + ["-c", path, "-o", obj]


def build(verbose: bool = False) -> str:
    """Compile every source and link libpkm.so; returns the library path."""
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        raise RuntimeError("hipcc not found")
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    for src in SOURCES:
        cmd = _compile_cmd(src)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and "is not a recognized feature" not in l]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("compile failed:\n" + "\n".join(f"--- {s}\n{o}" for s, o in failed))
    objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, LIB)
    return LIB


SAN_LIB = os.path.join(BUILD, "libpkm_san.so")
HOST_SOURCES = ["plan.hip", "runtime.hip", "host_math.cpp"]
# host-side sanitizers only: each -fsanitize goes to the host compilation through -Xarch_host
SAN_HIP = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_CXX = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def sanitizer_runtime() -> str:
    """The shared AddressSanitizer runtime of the ROCm clang (preloaded into the interpreter)."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang AddressSanitizer runtime not found")
    return hits[-1]


def build_sanitized(verbose: bool = False) -> str:
    """The library with its host code (plan, runtime, host math: every C-ABI entry point's
    argument checking and host arithmetic) under AddressSanitizer and UndefinedBehaviorSanitizer,
    linked with the kernel objects of the normal build (run build() first).  Writes
    libpkm_san.so into the build folder and returns its path; load it with the runtime of
    sanitizer_runtime() preloaded.  Device code is never built with a sanitizer."""
    objs = []
    procs = []
    for src in HOST_SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + "_san.o")
        if src.endswith(".hip"):
            cmd = [HIPCC] + DEVICE + COMMON + SAN_HIP + ["-c", path, "-o", obj]
        else:
            cmd = ["/opt/rocm/llvm/bin/clang++"] + COMMON + SAN_CXX + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = [(src, p.communicate()[0]) for src, p in procs]
    failed = [(src, out) for (src, out), (_, p) in zip(failed, procs) if p.returncode != 0]
    if failed:
        raise RuntimeError("sanitized compile failed:\n" + "\n".join(f"--- {s}\n{o}" for s, o in failed))
    kernels = [os.path.join(BUILD, s) for s in ("kernels_paint.o", "kernels_fft.o")]
    for k in kernels:
        if not os.path.exists(k):
            raise RuntimeError(f"{k} missing: run build() first")
    link = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-shared-libasan"] + SAN_HIP + \
        ["-o", SAN_LIB] + objs + kernels + ["-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n" + r.stdout)
    return SAN_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
