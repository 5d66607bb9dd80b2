"""Build the HIP library libpcprop.so for gfx950 (in-tree).

    python -m paper_2301_03989_amd.build

Compiles every ``csrc/*.hip`` with hipcc into ``paper_2301_03989_amd/libpcprop.so``.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libpcprop.so")
ARCH = os.environ.get("PCPROP_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def _deps():
    return sources() + sorted(glob.glob(os.path.join(PKG, "csrc", "*.h"))) + \
        [os.path.join(ROOT, "include", "pcprop.h")]


def source_hash() -> str:
    """sha256 over the sources the library is built from (names and contents)."""
    import hashlib
    h = hashlib.sha256()
    for f in _deps():
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(PKG, "csrc"), *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (res.stdout + res.stderr).splitlines()
            if "packed-fp32-ops" not in l and l.strip()]
    if res.returncode != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError("hipcc failed building libpcprop.so")
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    with open(LIB + ".srchash", "w") as fh:   # what the library was built from
        fh.write(source_hash() + "\n")
    return LIB


def is_stale() -> bool:
    """True when no library is built or its sources have changed since (by content, so
    that copies of the tree whose file times differ agree)."""
    if not os.path.exists(LIB):
        return True
    try:
        with open(LIB + ".srchash") as fh:
            return fh.read().strip() != source_hash()
    except OSError:
        t = os.path.getmtime(LIB)
        return any(os.path.getmtime(d) > t for d in _deps())


def ensure_built() -> str:
    """Build if no library exists or a source is newer than it (tests, smoke and bench
    otherwise load what is built)."""
    if is_stale():
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
