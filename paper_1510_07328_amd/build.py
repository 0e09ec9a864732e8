"""Build liblbm.so (HIP, gfx950) in-tree, under paper_1510_07328_amd/_build/.

Beside the library, liblbm.so.sources holds the sha256 of the sources and flags
it was built from; the binding rebuilds a library whose digest differs from the
sources in the tree, so a stale build is never loaded.

Every HIP source is compiled for gfx950 only, with packed FP32 instructions
disabled (-target-feature -packed-fp32-ops), without floating-point contraction
(fused multiply-adds are written out in the kernels, so the arithmetic is fixed
by the source), and C++17.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "liblbm.so")

SOURCES = ["coeffs.cpp", "lbm_kernels.hip", "lbm_capi.hip", "lbm_batch.hip", "lbm_batch_capi.hip", "srg_kernels.hip",
           "srg_capi.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# Host code under AddressSanitizer and UndefinedBehaviorSanitizer (build_sanitized);
# every sanitizer flag is scoped to the host compilation.
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-g"]
BUILD_SANITIZED = os.path.join(HERE, "_build_sanitized")
LIB_SANITIZED = os.path.join(BUILD_SANITIZED, "liblbm.so")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


STAMP = LIB + ".sources"


def source_digest() -> str:
    """sha256 over every file the library is built from (csrc/, include/) and the
    compiler flags, in a fixed order."""
    import hashlib

    h = hashlib.sha256(" ".join(HIPCC_FLAGS).encode())
    files = [os.path.join(CSRC, f) for f in os.listdir(CSRC)]
    inc = os.path.join(ROOT, "include")
    files += [os.path.join(inc, f) for f in os.listdir(inc)]
    for f in sorted(files, key=lambda p: os.path.relpath(p, ROOT)):
        if os.path.isfile(f):
            h.update(os.path.relpath(f, ROOT).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def built_digest():
    """Digest of the sources the present liblbm.so was built from (None if unknown)."""
    try:
        with open(STAMP) as fh:
            return fh.read().strip()
    except OSError:
        return None


def is_current() -> bool:
    return os.path.exists(LIB) and built_digest() == source_digest()


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    for src in sources():
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [cc, *HIPCC_FLAGS, *inc, "-c", *lang, src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
        if len(procs) >= jobs:
            p, s = procs.pop(0)
            if p.wait():
                raise RuntimeError(f"compile failed: {s}")
    for p, s in procs:
        if p.wait():
            raise RuntimeError(f"compile failed: {s}")
    digest = source_digest()  # of the sources as they were compiled
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    with open(STAMP + ".tmp", "w") as fh:
        fh.write(digest + "\n")
    os.replace(STAMP + ".tmp", STAMP)
    return LIB


def build_sanitized(verbose: bool = False, jobs: int = 4) -> str:
    """liblbm.so with its host code (argument checks, workspace layout, the float64
    coefficient construction, the launch wrappers) built under AddressSanitizer
    and UndefinedBehaviorSanitizer; the device code is compiled as usual.  The
    sanitizer runtime is not linked in; the process that loads the library
    preloads it.  Skipped when the build at hand was made from these sources."""
    stamp = LIB_SANITIZED + ".sources"
    digest = source_digest() + " " + " ".join(SANITIZE_HOST)
    try:
        with open(stamp) as fh:
            if os.path.exists(LIB_SANITIZED) and fh.read().strip() == digest:
                return LIB_SANITIZED
    except OSError:
        pass
    os.makedirs(BUILD_SANITIZED, exist_ok=True)
    cc = hipcc()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    for src in sources():
        obj = os.path.join(BUILD_SANITIZED, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [cc, *HIPCC_FLAGS, *SANITIZE_HOST, *inc, "-c", *lang, src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
        if len(procs) >= jobs:
            p, s = procs.pop(0)
            if p.wait():
                raise RuntimeError(f"compile failed: {s}")
    for p, s in procs:
        if p.wait():
            raise RuntimeError(f"compile failed: {s}")
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB_SANITIZED, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    with open(stamp, "w") as fh:
        fh.write(digest + "\n")
    return LIB_SANITIZED


if __name__ == "__main__":
    if "--sanitized" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
