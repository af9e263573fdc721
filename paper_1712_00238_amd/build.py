"""Compile the HIP sources into libsdfdock.so for gfx950 (in-tree).

Usage: python -m paper_1712_00238_amd.build [--jobs J] [--debug]
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsdfdock.so")
ARCH = os.environ.get("SDF_OFFLOAD_ARCH", "gfx950")

SOURCES = ["abi.cpp", "kernels_sdf.hip", "kernels_plain.hip", "kernels_fused.hip", "kernels_grad.hip",
           "kernels_topk.hip", "kernels_nfft.hip", "kernels_scan.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags(debug: bool = False) -> list:
    f = ["-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
         # keep the compiler from emitting packed FP32 arithmetic
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wno-unused-command-line-argument"]
    f += ["-O1", "-g"] if debug else ["-O3"]
    return f


def compile_one(src: str, debug: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    srcp = os.path.join(CSRC, src)
    deps = [srcp] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")] + \
        [os.path.join(ROOT, "include", "sdfdock.h")]
    if os.path.exists(obj) and all(os.path.getmtime(obj) >= os.path.getmtime(d) for d in deps):
        return obj
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [hipcc()] + flags(debug) + lang + ["-c", srcp, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(jobs: int = 6, debug: bool = False, force: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    if force:
        for f in os.listdir(BUILD):
            os.remove(os.path.join(BUILD, f))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: compile_one(s, debug), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC"] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


SAN_LIB = os.path.join(BUILD, "libsdfdock_hostsan.so")


def sanitizer_runtime() -> str:
    """The shared AddressSanitizer runtime of the ROCm clang (to preload into a
    process that loads the sanitized library)."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang AddressSanitizer runtime not found")
    return hits[-1]


def build_host_sanitized() -> str:
    """The ABI layer (abi.cpp) with AddressSanitizer and UndefinedBehavior-
    Sanitizer on its host code only (-Xarch_host: device code is not
    instrumented), linked with the kernel objects of the normal build, into
    _build/libsdfdock_hostsan.so.  For the CPU-side argument-validation tests;
    build() must have run first."""
    objs = [os.path.join(BUILD, os.path.splitext(f)[0] + ".o") for f in SOURCES if f != "abi.cpp"]
    if not all(os.path.exists(o) for o in objs):
        raise RuntimeError("kernel objects missing: run build() first")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    abi_o = os.path.join(BUILD, "abi_hostsan.o")
    cmd = [hipcc()] + flags() + san + ["-x", "hip", "-c", os.path.join(CSRC, "abi.cpp"), "-o", abi_o]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: abi.cpp (sanitized)\n{r.stderr}")
    clang = os.path.join(os.path.dirname(hipcc()), "..", "llvm", "bin", "clang++")
    link = [clang, "-shared", "-fPIC", "-fsanitize=address,undefined", abi_o] + objs + \
        ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", SAN_LIB]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed (sanitized)\n{' '.join(link)}\n{r.stderr}")
    return SAN_LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("--force", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.debug, a.force))


if __name__ == "__main__":
    sys.exit(main())
