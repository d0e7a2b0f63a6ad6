"""Builds the HIP library ``libnmfbeta.so`` in place (gfx950, hipcc)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libnmfbeta.so")
OBJDIR = os.path.join(PKG, "_build")

# Packed-FP32 instructions are disabled for all device code.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def build_library(verbose: bool = False) -> str:
    """Compiles every csrc/*.hip file and links libnmfbeta.so; returns its path."""
    hipcc = _hipcc()
    os.makedirs(OBJDIR, exist_ok=True)
    objs = []

    def compile_one(src):
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
        if verbose and out.strip():
            print(out, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, sources()))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


# Host-side sanitizer build: the host code compiled with AddressSanitizer and
# UndefinedBehaviorSanitizer (the device code unoptimized and uninstrumented,
# only so that the library links), linked against the shared sanitizer
# runtime, which the loading process must preload.  For the CPU tests of the
# host code; never loaded on a GPU.
SAN_DIR = os.path.join(OBJDIR, "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "libnmfbeta_san.so")
SAN_FLAGS = [
    "--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-g0", "-Xarch_host", "-g", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
    "-I" + INCLUDE, "-I" + CSRC,
]


def sanitizer_runtime() -> str:
    """Path of the shared AddressSanitizer runtime of ROCm's clang ('' if absent)."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else ""


def build_sanitized() -> str:
    """Builds the host-side sanitizer library (skipped when it is newer than
    every source and header); returns its path."""
    hipcc = _hipcc()
    os.makedirs(SAN_DIR, exist_ok=True)
    deps = sources() + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps.append(os.path.join(INCLUDE, "nmf_beta.h"))
    if os.path.exists(SAN_LIB) and os.path.getmtime(SAN_LIB) > max(os.path.getmtime(d) for d in deps):
        return SAN_LIB

    def compile_one(src):
        obj = os.path.join(SAN_DIR, os.path.basename(src) + ".o")
        r = subprocess.run([hipcc, *SAN_FLAGS, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("sanitizer compile failed for %s:\n%s" % (src, r.stdout + r.stderr))
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, sources()))
    clangxx = "/opt/rocm/llvm/bin/clang++"
    tmp = SAN_LIB + ".tmp"
    cmd = [clangxx, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libsan", "--hip-link",
           "--offload-arch=gfx950", *objs,
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitizer link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized())
    else:
        print(build_library(verbose=True))
