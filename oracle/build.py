"""Compile the C part of the oracle (TEST INFRASTRUCTURE ONLY) into oracle/_build/.

Built with plain gcc, -O2 -ffp-contract=off (no fused multiply-add, so every
rounding is the one the source spells out) and OpenMP over rows.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "liblbm_oracle.so")


SOURCES = ["lbm_oracle.c", "lbm_oracle_api.c"]  # lbm_oracle.h is included by both
FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall"]
STAMP = LIB + ".sources"


def source_digest() -> str:
    """sha256 of the C sources and flags (a library built from other sources is rebuilt)."""
    import hashlib

    h = hashlib.sha256(" ".join(FLAGS).encode())
    for name in SOURCES + ["lbm_oracle.h"]:
        with open(os.path.join(HERE, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()


def is_current() -> bool:
    try:
        with open(STAMP) as fh:
            return os.path.exists(LIB) and fh.read().strip() == source_digest()
    except OSError:
        return False


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    digest = source_digest()
    tmp = LIB + ".tmp"
    cmd = ["gcc", *FLAGS, "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    with open(STAMP + ".tmp", "w") as fh:
        fh.write(digest + "\n")
    os.replace(STAMP + ".tmp", STAMP)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
