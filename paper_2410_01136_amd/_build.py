"""Builds the HIP library libsynmarch.so for gfx950, in-tree.

Every .hip file under csrc/ is compiled to an object with hipcc and linked
into one shared library next to this file.  Packed FP32 instructions are
switched off for all device code.

build(sanitize=True) makes a second copy, libsynmarch_san.so, whose host code
(argument checks, prefactors, launch logic) is instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer (device code is compiled as
usual); it needs the clang ASan runtime preloaded into the process that loads
it (see asan_runtime()).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsynmarch.so")
LIB_SAN = os.path.join(HERE, "libsynmarch_san.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("SYNMARCH_ARCH", "gfx950")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
         "-I", os.path.join(HERE, "..", "include")]
# host-only instrumentation: each sanitizer flag is scoped to the host pass
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-g"]
SAN_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-shared-libsan"]


def asan_runtime() -> str:
    """Path of the clang ASan runtime that a process must preload to load the
    sanitized library (or the sanitized oracle)."""
    r = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                       text=True, check=True)
    return r.stdout.strip()


def build_id() -> str:
    """Hash of the library's sources (csrc/ and the public header); compiled in as
    the build id that keys the autotuner's cache."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*"))) + [os.path.join(HERE, "..", "include", "synmarch.h")]:
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _compile(src: str, sanitize: bool, bid: str) -> str:
    sub = "san" if sanitize else ""
    obj = os.path.join(BUILD_DIR, sub, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if sanitize else []), f'-DSYN_BUILD_ID="{bid}"', "-c", src,
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    os.makedirs(os.path.join(BUILD_DIR, "san" if sanitize else ""), exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    bid = build_id()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize, bid), srcs))
    lib = LIB_SAN if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *(SAN_LINK if sanitize else []),
           *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
