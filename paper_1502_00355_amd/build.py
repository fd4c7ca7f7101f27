"""Builds libsmartlap.so (HIP, gfx950) in-tree.

    python -m paper_1502_00355_amd.build

Every HIP source is compiled with contraction off (the quality and centroid
arithmetic must be one rounded operation per written operation), without
fast-math, and with packed FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsmartlap.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "smartlap.h")
DIGEST = LIB + ".srcsha"   # digest of the sources the library was built from
ARCH = os.environ.get("SMARTLAP_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-fno-fast-math",
    "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def source_digest() -> str:
    """sha256 over the name and contents of every file under csrc/ and of the
    public header."""
    h = hashlib.sha256()
    paths = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))] + [HEADER]
    for p in paths:
        if os.path.isfile(p):
            h.update(os.path.basename(p).encode() + b"\0")
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, p.stdout))
    # hipcc's host pass does not know the packed-fp32 feature; that warning is expected
    msgs = [ln for ln in p.stdout.splitlines() if ln.strip() and "packed-fp32-ops" not in ln]
    if msgs:
        sys.stderr.write("\n".join(msgs) + "\n")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout)
    digest = source_digest()
    os.replace(tmp, LIB)
    with open(DIGEST, "w") as f:
        f.write(digest + "\n")
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
