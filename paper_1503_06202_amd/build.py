"""Build the X-engine's HIP library ``libxeng.so`` in-tree for gfx950.

The library is one shared object from the HIP kernels and the C ABI in
``csrc/``; it exports the entry points declared in ``include/xeng.h``.  The
benchmark's MFMA-ceiling probe (``csrc/mfma_ceiling.hip``) is built beside it
as the executable ``mfma_ceiling``; it is a measurement tool, not part of the
library.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libxeng.so")
CEILING = os.path.join(PKG, "mfma_ceiling")
SOURCES = ("xcorr_plain.hip", "xcorr_chan.hip", "xcorr_gated.hip", "xcorr_batch.hip",
           "xcorr_wide.hip", "xeng_flags.hip", "xeng_beam.hip", "xeng_shift.hip",
           "xeng_noalloc.hip", "xeng_api.cpp")
OBJDIR = os.path.join(PKG, "_build")
ARCH = "gfx950"


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    p = os.path.join(rocm, "bin", "hipcc")
    return p if os.path.exists(p) else "hipcc"


FLAGS = [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
         # keep the compiler from emitting packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def object_path(src: str) -> str:
    return os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")


def compile_command(src: str) -> list:
    """One translation unit to an object (the units build in parallel)."""
    return [hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", object_path(src)]


def link_command(out: str = LIB) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + \
        [object_path(s) for s in SOURCES]


def ceiling_command(out: str = CEILING) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-o", out, os.path.join(CSRC, "mfma_ceiling.hip")]


def _run(cmd: list, what: str, quiet: bool) -> None:
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msg = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if noise not in l)
    if res.returncode != 0:
        sys.stderr.write(msg + "\n")
        raise RuntimeError(f"{what} build failed: " + " ".join(cmd))
    if msg.strip() and not quiet:
        print(msg)


# Host-side sanitizer build of the C ABI (argument checks, plans, work lists):
# xeng_api.cpp is compiled with AddressSanitizer and UndefinedBehaviorSanitizer
# for the host only and linked with the ordinary kernel objects into
# _build/libxeng_san.so.  Load it with XENG_LIBRARY pointing at it and clang's
# ASan runtime preloaded (asan_runtime()).
SAN_LIB = os.path.join(OBJDIR, "libxeng_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
             "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """clang's shared AddressSanitizer runtime (to preload for libxeng_san.so)."""
    res = subprocess.run([hipcc(), "--print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
        import glob

        hits = glob.glob(os.path.join(rocm, "lib/llvm/lib/clang/*/lib/*/libclang_rt.asan-x86_64.so"))
        hits += glob.glob(os.path.join(rocm, "llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
        path = hits[0] if hits else ""
    return path


def build_sanitized(quiet: bool = True) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    for src in SOURCES:
        if src != "xeng_api.cpp" and not os.path.exists(object_path(src)):
            _run(compile_command(src), src, quiet)
    san_obj = os.path.join(OBJDIR, "xeng_api_san.o")
    _run([hipcc()] + FLAGS + SAN_FLAGS + ["-c", os.path.join(CSRC, "xeng_api.cpp"), "-o", san_obj],
         "xeng_api.cpp (sanitized)", quiet)
    objs = [object_path(s) for s in SOURCES if s != "xeng_api.cpp"] + [san_obj]
    tmp = SAN_LIB + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan", "-Xarch_host",
          "-fsanitize=address,undefined", "-o", tmp] + objs, "libxeng_san", quiet)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def build(quiet: bool = True, jobs: int = 0) -> str:
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, compile_command(s), s, quiet) for s in SOURCES]:
            f.result()
    tmp = LIB + ".tmp"
    _run(link_command(tmp), "libxeng", quiet)
    os.replace(tmp, LIB)
    tmp = CEILING + ".tmp"
    _run(ceiling_command(tmp), "mfma_ceiling", quiet)
    os.replace(tmp, CEILING)
    if not quiet:
        print("built", LIB)
        print("built", CEILING)
    return LIB


if __name__ == "__main__":
    build(quiet=False)
