"""Build the gfx950 shared library ``libtfsph.so`` in-tree with hipcc.

Usage: ``python -m paper_1908_01682_amd.build`` (or ``build()`` from Python).
The library has no PyTorch dependency: it exports the C ABI of
``include/tfsph.h`` and links only the HIP runtime.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtfsph.so")
SOURCES = [os.path.join(CSRC, f) for f in ("tfsph.hip", "batch.hip", "adjoint.hip")]
HEADERS = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))] + \
    [os.path.join(ROOT, "include", "tfsph.h")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep contraction within single expressions so every kernel that shares a
    # device function rounds identically
    "-ffp-contract=on",
    # no packed-FP32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-result",
]


def build(verbose: bool = True) -> str:
    """Compile every HIP source of the package into libtfsph.so (always rebuilds).

    Each source is compiled to an object in its own hipcc process (they run
    concurrently), then the objects are linked into the shared library."""
    tag = f".tmp{os.getpid()}"
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(os.path.basename(src))[0] + tag + ".o")
        cmd = [hipcc()] + compile_flags + ["-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((obj, subprocess.Popen(cmd)))
    failed = [obj for obj, proc in jobs if proc.wait() != 0]
    objs = [obj for obj, _ in jobs]
    try:
        if failed:
            raise subprocess.CalledProcessError(1, "hipcc -c", f"failed: {failed}")
        tmp = LIB + tag
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    return LIB


def needs_build() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    build()
    sys.exit(0)
